// Append candidates after a fusion, for one stream: the depth surfels that
// fusion matched to no live surfel, skinned in the live frame (Sec. 6.2),
// tested for a compressive warp (Sec. 6.3) and for their distance from the
// nodes (Sec. 6.4), and warped back to the reference frame.
//
//   append_eval   one thread per depth pixel. A candidate (normal present,
//                 no fused surfel) takes the 4 nearest live node positions
//                 c_j = T_j p_j (FP32 key, ties to the lower index; the node
//                 positions pass through LDS in tiles). Node i stays in the
//                 set only if (1 - eps)^2 |p_i - p_0|^2 < |c_i - c_0|^2 <
//                 (1 + eps)^2 |p_i - p_0|^2 (Eq. 7 on squares, FP32); the
//                 nearest always stays. The candidate is far if the plain
//                 Gaussian weight sum of the kept nodes is below delta_nn.
//                 Otherwise its reference position is R^T (V - t) of the
//                 normalised blend of the kept nodes (weights evaluated at
//                 V), and the derivative of that map is taken by central
//                 differences (step 1 mm, node set fixed, weights re-evaluated
//                 at each offset point); the candidate is compressive if the
//                 largest eigenvalue of F^T F exceeds (1 + eps)^2 (Eq. 8,
//                 largest singular value of F above 1 + eps). Survivors get a
//                 flag; the counts are summed per wave, one atomic each.
//   append_write  after an exclusive scan of the flags: survivor k (in
//                 row-major pixel order) writes its pixel, reference position
//                 and normal, and the depth surfel's radius and confidence
//                 (Sec. 5), up to the caller's capacity.
//   keep_mark, compact_surfels   the geometry update: flags of the existing
//                 surfels that stay, then (after a scan) the kept surfels and
//                 the appended ones copied into fresh caller-order arrays.
#include "swgn_fusion.h"
#include "swgn_impl.h"
#include "swgn_launch.h"

namespace swgn {

namespace {

constexpr int kAppendTile = 1024;      // live node positions staged per pass
constexpr float kFdStep = 1e-3f;       // central-difference step of Eq. 8

// Reference position (and normal) of live point x through the inverse of the
// normalised blend of the kept nodes, weights exp(-(|x - c_j|^2 - |x - c_0|^2)
// / (2 sigma^2)) normalised over the kept nodes.
__device__ __forceinline__ float3 warp_back(float3 x, float3* nrm, const int (&id)[4], const bool (&kp)[4],
                                            const float4* __restrict__ cl, const float4* __restrict__ dq,
                                            float inv2s2) {
    float kd[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float4 c = cl[id[k]];
        const float dx = x.x - c.x, dy = x.y - c.y, dz = x.z - c.z;
        kd[k] = (dx * dx + dy * dy) + dz * dz;
    }
    float e[4];
    e[0] = 1.0f;
#pragma unroll
    for (int k = 1; k < 4; ++k) e[k] = kp[k] ? expf(-(kd[k] - kd[0]) * inv2s2) : 0.f;
    const float inv = 1.0f / (((e[0] + e[1]) + e[2]) + e[3]);
    const Warp wp = warp_surfel(make_int4(id[0], id[1], id[2], id[3]),
                                make_float4(e[0] * inv, e[1] * inv, e[2] * inv, e[3] * inv), x,
                                nrm ? *nrm : make_float3(0.f, 0.f, 0.f), dq);
    const float3 u3 = make_float3(-wp.cr.x, -wp.cr.y, -wp.cr.z);     // conjugate rotation
    const float3 tb = scale3(vec_mul_conj(wp.cd, wp.cr), 2.0f);
    if (nrm) *nrm = qrot(wp.cr.w, u3, *nrm);
    return qrot(wp.cr.w, u3, sub3(x, tb));
}

// Largest eigenvalue of the symmetric 3x3 matrix M (Smith's trigonometric
// closed form: M = q I + p B, lambda = q + 2 p cos(acos(det(B) / 2) / 3)).
__device__ __forceinline__ float max_eig_sym3(float m00, float m01, float m02, float m11, float m12, float m22) {
    const float p1 = (m01 * m01 + m02 * m02) + m12 * m12;
    const float q = ((m00 + m11) + m22) * (1.0f / 3.0f);
    const float a = m00 - q, b = m11 - q, c = m22 - q;
    const float p2 = ((a * a + b * b) + c * c) + 2.0f * p1;
    if (!(p2 > 0.f)) return q;
    const float p = sqrtf(p2 * (1.0f / 6.0f));
    const float ip = 1.0f / p;
    const float b00 = a * ip, b11 = b * ip, b22 = c * ip, b01 = m01 * ip, b02 = m02 * ip, b12 = m12 * ip;
    const float det = b00 * (b11 * b22 - b12 * b12) - b01 * (b01 * b22 - b12 * b02) + b02 * (b01 * b12 - b11 * b02);
    const float r = fminf(fmaxf(0.5f * det, -1.0f), 1.0f);
    return q + 2.0f * p * cosf(acosf(r) * (1.0f / 3.0f));
}

__global__ void __launch_bounds__(256) k_append_eval(AppendArgs a) {
    __shared__ float4 tile[kAppendTile];
    __shared__ int tid[kAppendTile];
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int npx = a.cam.W * a.cam.H;
    const bool in = u < npx;
    const float4 nm = in ? a.nmap[u] : make_float4(0.f, 0.f, 0.f, 0.f);
    const bool cand = in && nm.w > 0.f && a.match[u] < 0;
    const int x = in ? u % a.cam.W : 0, y = in ? u / a.cam.W : 0;
    const float d = nm.w;
    const float3 V = make_float3((((float)x - a.cam.cx) / a.cam.fx) * d, (((float)y - a.cam.cy) / a.cam.fy) * d, d);
    float kd[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
    int ki[4] = {0, 0, 0, 0};
    for (int base = 0; base < a.nn; base += kAppendTile) {
        const int cnt = min(kAppendTile, a.nn - base);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
            tile[t] = a.cl[base + t];
            tid[t] = a.node_id[base + t];
        }
        __syncthreads();
        if (cand) {
            for (int t = 0; t < cnt; ++t) {
                const float4 c = tile[t];
                const float dx = V.x - c.x, dy = V.y - c.y, dz = V.z - c.z;
                knn_insert_lex<4>(kd, ki, (dx * dx + dy * dy) + dz * dz, tid[t]);
            }
        }
    }
    // the nearest set, found in the caller's node numbering (ties to the
    // lower caller index), back in the library's
#pragma unroll
    for (int k = 0; k < 4; ++k) ki[k] = cand ? a.node_inv[ki[k]] : 0;
    bool far = false, comp = false;
    float3 vr = make_float3(0.f, 0.f, 0.f), nr = make_float3(0.f, 0.f, 0.f);
    if (cand) {
        // Eq. 7 on squares
        bool kp[4] = {true, false, false, false};
        const float4 c0 = a.cl[ki[0]];
        const float4 p0 = a.pref[ki[0]];
        const float lo = 1.0f - a.eps, hi = 1.0f + a.eps;
#pragma unroll
        for (int k = 1; k < 4; ++k) {
            const float4 c = a.cl[ki[k]];
            const float4 p = a.pref[ki[k]];
            const float lx = c.x - c0.x, ly = c.y - c0.y, lz = c.z - c0.z;
            const float rx = p.x - p0.x, ry = p.y - p0.y, rz = p.z - p0.z;
            const float dl = (lx * lx + ly * ly) + lz * lz;
            const float dr = (rx * rx + ry * ry) + rz * rz;
            kp[k] = (lo * lo * dr < dl) && (dl < hi * hi * dr);
        }
        // weight sum of the kept nodes (Sec. 6.4)
        float S = expf(-kd[0] * a.inv2s2);
#pragma unroll
        for (int k = 1; k < 4; ++k) S += kp[k] ? expf(-kd[k] * a.inv2s2) : 0.f;
        far = !(S >= a.delta_nn);
        if (!far) {
            float3 n = make_float3(nm.x, nm.y, nm.z);
            vr = warp_back(V, &n, ki, kp, a.cl, a.dq, a.inv2s2);
            nr = n;
            // d x_ref / d x_live by central differences (Eq. 8)
            float F[3][3];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                float3 xp = V, xm = V;
                if (ax == 0) { xp.x += kFdStep; xm.x -= kFdStep; }
                if (ax == 1) { xp.y += kFdStep; xm.y -= kFdStep; }
                if (ax == 2) { xp.z += kFdStep; xm.z -= kFdStep; }
                const float den = ax == 0 ? xp.x - xm.x : (ax == 1 ? xp.y - xm.y : xp.z - xm.z);
                const float3 rp = warp_back(xp, nullptr, ki, kp, a.cl, a.dq, a.inv2s2);
                const float3 rm = warp_back(xm, nullptr, ki, kp, a.cl, a.dq, a.inv2s2);
                const float id = 1.0f / den;
                F[0][ax] = (rp.x - rm.x) * id;
                F[1][ax] = (rp.y - rm.y) * id;
                F[2][ax] = (rp.z - rm.z) * id;
            }
            float m[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) m[i][j] = (F[0][i] * F[0][j] + F[1][i] * F[1][j]) + F[2][i] * F[2][j];
            const float lam = max_eig_sym3(m[0][0], m[0][1], m[0][2], m[1][1], m[1][2], m[2][2]);
            comp = lam > hi * hi;
        }
    }
    const bool ok = cand && !far && !comp;
    // wave sums of the counts, one atomic per wave and count
    const unsigned long long bc = __ballot(cand), bf = __ballot(cand && far), bm = __ballot(comp);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (bc) atomicAdd(&a.counts[0], __popcll(bc));
        if (bf) atomicAdd(&a.counts[1], __popcll(bf));
        if (bm) atomicAdd(&a.counts[2], __popcll(bm));
    }
    if (!in) return;
    a.flag[u] = ok ? 1 : 0;
    if (ok) {
        a.sv[u] = make_float4(vr.x, vr.y, vr.z, 0.f);
        a.sn[u] = make_float4(nr.x, nr.y, nr.z, 0.f);
    }
}

__global__ void __launch_bounds__(256) k_append_write(AppendArgs a, const int* __restrict__ pos) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int npx = a.cam.W * a.cam.H;
    if (u >= npx || !a.flag[u]) return;
    const int k = pos[u];
    if (k >= a.max_out) return;
    const int x = u % a.cam.W, y = u / a.cam.W;
    const float4 nm = a.nmap[u];
    const float4 v = a.sv[u], n = a.sn[u];
    // the depth surfel's confidence and radius (Sec. 5), as fusion takes them
    const float gx = (float)x - a.cam.cx, gy = (float)y - a.cam.cy;
    const float gamma2 = (gx * gx + gy * gy) / (a.cam.cx * a.cam.cx + a.cam.cy * a.cam.cy);
    a.out_pixel[k] = u;
    a.out_pos[3 * (int64_t)k + 0] = v.x; a.out_pos[3 * (int64_t)k + 1] = v.y; a.out_pos[3 * (int64_t)k + 2] = v.z;
    a.out_nrm[3 * (int64_t)k + 0] = n.x; a.out_nrm[3 * (int64_t)k + 1] = n.y; a.out_nrm[3 * (int64_t)k + 2] = n.z;
    a.out_conf[k] = expf(-gamma2 / (2.0f * kFusePhi * kFusePhi));
    a.out_rad[k] = 1.41421356237f * nm.w / (a.cam.fx * fmaxf(fabsf(nm.z), a.cos_max));
}

// Geometry update (Sec. 6.4): an existing surfel stays unless its confidence
// is below delta_stable more than t_low_confid frames after its t_init.
__global__ void __launch_bounds__(256) k_keep_mark(int ns, const float* __restrict__ conf,
                                                   const int* __restrict__ tinit, int t_now, float stable,
                                                   int t_low, int* __restrict__ flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ns) flag[i] = (conf[i] < stable && t_now - tinit[i] > t_low) ? 0 : 1;
}

// The updated arrays: kept surfel i at pos[i], appended surfel k at nkeep + k.
__global__ void __launch_bounds__(256) k_compact_surfels(CompactArgs c) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < c.ns) {
        if (!c.flag[i]) return;
        const int j = c.pos[i];
        for (int q = 0; q < 3; ++q) {
            c.dpos[3 * (int64_t)j + q] = c.spos[3 * (int64_t)i + q];
            c.dnrm[3 * (int64_t)j + q] = c.snrm[3 * (int64_t)i + q];
        }
        c.drad[j] = c.srad[i];
        c.dconf[j] = c.sconf[i];
        c.dtobs[j] = c.stobs[i];
        c.dtinit[j] = c.stinit[i];
    } else if (i < c.ns + c.napp) {
        const int k = i - c.ns, j = c.nkeep + k;
        for (int q = 0; q < 3; ++q) {
            c.dpos[3 * (int64_t)j + q] = c.apos[3 * (int64_t)k + q];
            c.dnrm[3 * (int64_t)j + q] = c.anrm[3 * (int64_t)k + q];
        }
        c.drad[j] = c.arad[k];
        c.dconf[j] = c.aconf[k];
        c.dtobs[j] = c.t_now;
        c.dtinit[j] = c.t_now;
    }
}

__global__ void __launch_bounds__(256) k_f4_to_positions(int n, const float4* __restrict__ in,
                                                         float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 p = in[i];
    out[3 * i + 0] = p.x;
    out[3 * i + 1] = p.y;
    out[3 * i + 2] = p.z;
}

}  // namespace

void launch_f4_to_positions(int n, const float4* in, float* out, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_f4_to_positions, dim3((n + 255) / 256), dim3(256), 0, st, n, in, out);
}

void launch_keep_mark(int ns, const float* conf, const int* tinit, int t_now, float stable, int t_low, int* flag,
                      hipStream_t st) {
    if (ns > 0)
        hipLaunchKernelGGL(k_keep_mark, dim3((ns + 255) / 256), dim3(256), 0, st, ns, conf, tinit, t_now, stable,
                           t_low, flag);
}

void launch_compact_surfels(const CompactArgs& c, hipStream_t st) {
    const int64_t n = (int64_t)c.ns + c.napp;
    if (n > 0) hipLaunchKernelGGL(k_compact_surfels, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, c);
}

void launch_append(const AppendArgs& a, int* pos, int* scan_tmp, hipStream_t st) {
    const int npx = a.cam.W * a.cam.H;
    const dim3 g((npx + 255) / 256);
    hipLaunchKernelGGL(k_append_eval, g, dim3(256), 0, st, a);
    exclusive_scan(a.flag, pos, npx + 1, scan_tmp, st);
    hipLaunchKernelGGL(k_append_write, g, dim3(256), 0, st, a, pos);
}

}  // namespace swgn
