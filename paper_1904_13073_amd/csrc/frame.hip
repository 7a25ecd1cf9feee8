// Per-frame kernels of the Gauss-Newton warp-field solve (Sec. 7), part 1:
//
//   depth_prep   normal map of the depth image (Sec. 5); resets the index map
//   clear_z      index-map reset
//   warp_zbuf    dual-quaternion warp of every surfel (Sec. 3, Eq. 1-2) and
//                a 64-bit atomic-min z-buffer of (z bits, surfel index) (Sec. 7)
//   corr_jac     projective correspondence, point-to-plane residual and its
//                exact Jacobian with respect to the 4 node twists
// plus node-state conversions and capture helpers. Assembly is in
// assemble.hip, the linear solve and node update in solve.hip.
//
// Sums are taken in a fixed order everywhere, so a frame solve is
// bit-reproducible run to run.
#include "swgn_impl.h"
#include "swgn_launch.h"

namespace swgn {

// ---------------------------------------------------------------------------
// Depth preprocessing: normal map by central differences (Sec. 5).
// nmap = (n, d) where the normal is defined, (0, 0, 0, 0) elsewhere.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_depth_prep(Cam cam, const float* __restrict__ depth, float gate,
                                                    float4* __restrict__ nmap, unsigned long long* __restrict__ zbuf,
                                                    int* __restrict__ flags) {
    int x = blockIdx.x * 16 + (threadIdx.x & 15);
    int y = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 4) flags[threadIdx.x] = 0;
    if (x >= cam.W || y >= cam.H) return;
    int W = cam.W;
    zbuf[y * W + x] = ~0ull;   // index map of the first iteration
    float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
    if (x > 0 && y > 0 && x < cam.W - 1 && y < cam.H - 1) {
        float dc = depth[y * W + x];
        float dU = depth[(y - 1) * W + x], dD = depth[(y + 1) * W + x];
        float dL = depth[y * W + x - 1], dR = depth[y * W + x + 1];
        bool ok = depth_ok(dc) && depth_ok(dU) && depth_ok(dD) && depth_ok(dL) && depth_ok(dR);
        if (ok) {
            ok = fabsf(dU - dc) <= gate && fabsf(dD - dc) <= gate && fabsf(dL - dc) <= gate &&
                 fabsf(dR - dc) <= gate;
        }
        if (ok) {
            float3 vU = backproject(cam, x, y - 1, dU), vD = backproject(cam, x, y + 1, dD);
            float3 vL = backproject(cam, x - 1, y, dL), vR = backproject(cam, x + 1, y, dR);
            float3 a = sub3(vD, vU);   // V(x, y+1) - V(x, y-1)
            float3 b = sub3(vR, vL);   // V(x+1, y) - V(x-1, y)
            float c0 = a.y * b.z - a.z * b.y;
            float c1 = a.z * b.x - a.x * b.z;
            float c2 = a.x * b.y - a.y * b.x;
            float nn = (c0 * c0 + c1 * c1) + c2 * c2;
            if (nn > 0.f && nn < INFINITY) {
                float ln = sqrtf(nn);
                float n0 = c0 / ln, n1 = c1 / ln, n2 = c2 / ln;
                float3 vc = backproject(cam, x, y, dc);
                float dt = (n0 * vc.x + n1 * vc.y) + n2 * vc.z;
                if (dt > 0.f) { n0 = -n0; n1 = -n1; n2 = -n2; }
                out = make_float4(n0, n1, n2, dc);
            }
        }
    }
    nmap[y * W + x] = out;
}

__global__ void k_clear_z(unsigned long long* __restrict__ z, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = ~0ull;
}

struct SurfelArrays {
    const float *px, *py, *pz, *nx, *ny, *nz;
    const int4* idx;
    const float4* w;
    const int* orig;
};

__device__ __forceinline__ unsigned long long zkey(float z, int orig) {
    return ((unsigned long long)__float_as_uint(z) << 32) | (unsigned long long)(unsigned)orig;
}

// ---------------------------------------------------------------------------
// Warp + index map
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_warp_zbuf(int ns, SurfelArrays s, const float4* __restrict__ dq,
                                                   Cam cam, unsigned long long* __restrict__ zbuf) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns) return;
    float3 v = make_float3(s.px[i], s.py[i], s.pz[i]);
    Warp wp = warp_surfel(s.idx[i], s.w[i], v, make_float3(0.f, 0.f, 0.f), dq);
    if (!wp.ok) return;
    int ux, uy;
    if (!project(cam, wp.v, ux, uy)) return;
    atomicMin(&zbuf[uy * cam.W + ux], zkey(wp.v.z, s.orig[i]));
}

// ---------------------------------------------------------------------------
// Correspondence, residual and Jacobian
// ---------------------------------------------------------------------------
struct CorrOut {
    float* J;              // [pitch][32]: 24 Jacobian entries (node position x 6), r, zero padding
    double* part_e;        // per block sum of r^2
    int* part_n;           // per block correspondence count
    int pitch;
    // capture (null unless this iteration is captured)
    int* corr_map;
    float* live_pos;
};

__global__ void __launch_bounds__(256) k_corr_jac(int ns, SurfelArrays s, const float4* __restrict__ dq,
        const float4* __restrict__ cl, Cam cam, const unsigned long long* __restrict__ zbuf,
        const float4* __restrict__ nmap, float dist2, float cosn, CorrOut o) {
    __shared__ double sh[40];
    __shared__ int shi[16];
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool live = i < ns;
    float r = 0.f;
    float Jw[4][3], Jt[4][3];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) { Jw[k][c] = 0.f; Jt[k][c] = 0.f; }
    bool matched = false;
    int4 id = make_int4(0, 0, 0, 0);
    int pix = 0, org = 0;
    Warp wp;
    wp.ok = false;
    if (live) {
        id = s.idx[i];
        org = s.orig[i];
        float3 v = make_float3(s.px[i], s.py[i], s.pz[i]);
        float3 n = make_float3(s.nx[i], s.ny[i], s.nz[i]);
        wp = warp_surfel(id, s.w[i], v, n, dq);
        int ux, uy;
        if (wp.ok && project(cam, wp.v, ux, uy)) {
            pix = uy * cam.W + ux;
            if (zbuf[pix] == zkey(wp.v.z, org)) {
                float4 nm = nmap[pix];
                if (nm.w > 0.f) {
                    float3 V = backproject(cam, ux, uy, nm.w);
                    float3 dv = sub3(wp.v, V);
                    float d2 = (dv.x * dv.x + dv.y * dv.y) + dv.z * dv.z;
                    float3 N = make_float3(nm.x, nm.y, nm.z);
                    if (d2 < dist2 && dot3(wp.n, N) > cosn) {
                        matched = true;
                        r = dot3(N, dv);
                        // d r / d xi_k, closed form of N^T dF/db(b; v) w_k s_k M(q_k, c_k)
                        Q4 Nq = {0.f, N.x, N.y, N.z};
                        Q4 P = qmul(Nq, wp.cr);
                        Q4 Qd = qmul(Nq, wp.cd);
                        Q4 PV = qmul(P, Q4{0.f, v.x, v.y, v.z});
                        float ndv = dot3(N, wp.v);
                        const int ids[4] = {id.x, id.y, id.z, id.w};
                        const float4 w4 = s.w[i];
                        const float wk[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            Q4 rk = q4(dq[2 * ids[k]]);
                            Q4 dk = q4(dq[2 * ids[k] + 1]);
                            float4 c4 = cl[ids[k]];
                            float3 ck = make_float3(c4.x, c4.y, c4.z);
                            float a = (wk[k] * wp.sgn[k]) * wp.inv_beta;
                            float3 h = vec_mul_conj(P, rk);
                            float3 g1 = vec_mul_conj(P, dk);
                            float3 g2 = vec_mul_conj(PV, rk);
                            float3 g3 = vec_mul_conj(Qd, rk);
                            float3 g4 = vec_mul_conj(wp.cr, rk);
                            float3 g5 = cross3(ck, h);
                            float3 gw = sub3(sub3(sub3(g1, g2), g3), add3(scale3(g4, ndv), g5));
                            Jw[k][0] = a * gw.x; Jw[k][1] = a * gw.y; Jw[k][2] = a * gw.z;
                            Jt[k][0] = a * h.x;  Jt[k][1] = a * h.y;  Jt[k][2] = a * h.z;
                        }
                    }
                }
            }
        }
    }
    if (live) {
        // one 128-byte row per surfel, node blocks by position within the
        // surfel's ascending node set, then the residual
        const int ids[4] = {id.x, id.y, id.z, id.w};
        float* row = o.J + (size_t)i * 32;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int pos = (ids[0] < ids[k]) + (ids[1] < ids[k]) + (ids[2] < ids[k]) + (ids[3] < ids[k]);
            float2* Jp = reinterpret_cast<float2*>(row + pos * 6);
            Jp[0] = make_float2(Jw[k][0], Jw[k][1]);
            Jp[1] = make_float2(Jw[k][2], Jt[k][0]);
            Jp[2] = make_float2(Jt[k][1], Jt[k][2]);
        }
        row[24] = r;
        if (o.live_pos) {
            float nanv = __int_as_float(0x7fc00000);
            o.live_pos[3 * org + 0] = wp.ok ? wp.v.x : nanv;
            o.live_pos[3 * org + 1] = wp.ok ? wp.v.y : nanv;
            o.live_pos[3 * org + 2] = wp.ok ? wp.v.z : nanv;
            if (matched) o.corr_map[pix] = org;
        }
    }
    double e = block_sum((double)r * (double)r, sh);
    int cnt = wave_sumi(matched ? 1 : 0);
    if ((threadIdx.x % kWave) == 0) shi[threadIdx.x / kWave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int c = 0;
        for (int q = 0; q < (int)(blockDim.x / kWave); ++q) c += shi[q];
        o.part_e[blockIdx.x] = e;
        o.part_n[blockIdx.x] = c;
    }
}

// Node state from [R | t] (FP64 conversion, w >= 0) and its tables.
__global__ void k_nodes_from_se3(int nn, const float* __restrict__ se3, const float4* __restrict__ pref,
                                 float4* __restrict__ rq, float4* __restrict__ tt, float4* __restrict__ dq,
                                 float4* __restrict__ cl) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nn) return;
    double m[12];
    if (se3) {
        for (int t = 0; t < 12; ++t) m[t] = (double)se3[12 * k + t];
    } else {
        for (int t = 0; t < 12; ++t) m[t] = 0.0;
        m[0] = m[5] = m[10] = 1.0;
    }
    double R00 = m[0], R01 = m[1], R02 = m[2], R10 = m[4], R11 = m[5], R12 = m[6], R20 = m[8], R21 = m[9],
           R22 = m[10];
    double tr = R00 + R11 + R22;
    double qw, qx, qy, qz;
    if (tr >= R00 && tr >= R11 && tr >= R22) {
        double s = 2.0 * sqrt(fmax(1.0 + tr, 0.0));
        qw = 0.25 * s; qx = (R21 - R12) / s; qy = (R02 - R20) / s; qz = (R10 - R01) / s;
    } else if (R00 >= R11 && R00 >= R22) {
        double s = 2.0 * sqrt(fmax(1.0 + R00 - R11 - R22, 0.0));
        qw = (R21 - R12) / s; qx = 0.25 * s; qy = (R01 + R10) / s; qz = (R02 + R20) / s;
    } else if (R11 >= R22) {
        double s = 2.0 * sqrt(fmax(1.0 - R00 + R11 - R22, 0.0));
        qw = (R02 - R20) / s; qx = (R01 + R10) / s; qy = 0.25 * s; qz = (R12 + R21) / s;
    } else {
        double s = 2.0 * sqrt(fmax(1.0 - R00 - R11 + R22, 0.0));
        qw = (R10 - R01) / s; qx = (R02 + R20) / s; qy = (R12 + R21) / s; qz = 0.25 * s;
    }
    double nq = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    if (qw < 0) nq = -nq;
    Q4 r = Q4{(float)(qw / nq), (float)(qx / nq), (float)(qy / nq), (float)(qz / nq)};
    float3 t = make_float3((float)m[3], (float)m[7], (float)m[11]);
    rq[k] = f4(r);
    tt[k] = make_float4(t.x, t.y, t.z, 0.f);
    node_tables(pref[k], r, t, dq, cl, k);
}

__global__ void k_node_se3_out(int nn, const float4* __restrict__ rq, const float4* __restrict__ tt,
                               float* __restrict__ out) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nn) return;
    float4 q = rq[k];
    double w = q.x, x = q.y, y = q.z, z = q.w;
    double n2 = w * w + x * x + y * y + z * z;
    double s = 2.0 / n2;
    float4 t = tt[k];
    float* o = out + 12 * k;
    o[0] = (float)(1 - s * (y * y + z * z)); o[1] = (float)(s * (x * y - w * z)); o[2] = (float)(s * (x * z + w * y));
    o[3] = t.x;
    o[4] = (float)(s * (x * y + w * z)); o[5] = (float)(1 - s * (x * x + z * z)); o[6] = (float)(s * (y * z - w * x));
    o[7] = t.y;
    o[8] = (float)(s * (x * z - w * y)); o[9] = (float)(s * (y * z + w * x)); o[10] = (float)(1 - s * (x * x + y * y));
    o[11] = t.z;
}

__global__ void k_export_index_map(int npx, const unsigned long long* __restrict__ z, int* __restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npx) return;
    unsigned long long v = z[i];
    out[i] = v == ~0ull ? -1 : (int)(unsigned)(v & 0xffffffffull);
}

__global__ void k_pointer_positions(int n, const float* __restrict__ pos, float4* __restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = make_float4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], 0.f);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
void launch_depth_prep(const Cam& cam, const float* depth, float gate, float4* nmap, unsigned long long* zbuf,
                       int* flags, hipStream_t st) {
    dim3 grid((cam.W + 15) / 16, (cam.H + 15) / 16);
    hipLaunchKernelGGL(k_depth_prep, grid, dim3(256), 0, st, cam, depth, gate, nmap, zbuf, flags);
}

void launch_clear_z(unsigned long long* z, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_clear_z, dim3((n + 255) / 256), dim3(256), 0, st, z, n);
}

void launch_warp_zbuf(int ns, const SurfelView& sv, const float4* dq, const Cam& cam, unsigned long long* z,
                      hipStream_t st) {
    SurfelArrays s{sv.px, sv.py, sv.pz, sv.nx, sv.ny, sv.nz, sv.idx, sv.w, sv.orig};
    hipLaunchKernelGGL(k_warp_zbuf, dim3((ns + 255) / 256), dim3(256), 0, st, ns, s, dq, cam, z);
}

int corr_blocks(int ns) { return (ns + 255) / 256; }

void launch_corr_jac(int ns, const SurfelView& sv, const float4* dq, const float4* cl, const Cam& cam,
                     const unsigned long long* z, const float4* nmap, float dist2, float cosn, float* J,
                     int pitch, double* part_e, int* part_n, int* corr_map, float* live_pos,
                     hipStream_t st) {
    SurfelArrays s{sv.px, sv.py, sv.pz, sv.nx, sv.ny, sv.nz, sv.idx, sv.w, sv.orig};
    CorrOut o{J, part_e, part_n, pitch, corr_map, live_pos};
    hipLaunchKernelGGL(k_corr_jac, dim3(corr_blocks(ns)), dim3(256), 0, st, ns, s, dq, cl, cam, z, nmap, dist2,
                       cosn, o);
}

void launch_nodes_from_se3(int nn, const float* se3, const float4* pref, float4* rq, float4* tt, float4* dq,
                           float4* cl, hipStream_t st) {
    hipLaunchKernelGGL(k_nodes_from_se3, dim3((nn + 255) / 256), dim3(256), 0, st, nn, se3, pref, rq, tt, dq, cl);
}

void launch_node_se3_out(int nn, const float4* rq, const float4* tt, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_node_se3_out, dim3((nn + 255) / 256), dim3(256), 0, st, nn, rq, tt, out);
}

void launch_export_index_map(int npx, const unsigned long long* z, int* out, hipStream_t st) {
    hipLaunchKernelGGL(k_export_index_map, dim3((npx + 255) / 256), dim3(256), 0, st, npx, z, out);
}

void launch_positions_to_f4(int n, const float* pos, float4* out, hipStream_t st) {
    hipLaunchKernelGGL(k_pointer_positions, dim3((n + 255) / 256), dim3(256), 0, st, n, pos, out);
}


}  // namespace swgn

namespace swgn {

__global__ void k_fill_i32(int* __restrict__ p, int n, int v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_tables_from_state(int nn, const float4* __restrict__ pref, const float4* __restrict__ rq,
                                    const float4* __restrict__ tt, float4* __restrict__ dq, float4* __restrict__ cl) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nn) return;
    float4 t = tt[k];
    node_tables(pref[k], q4(rq[k]), make_float3(t.x, t.y, t.z), dq, cl, k);
}

void launch_fill_i32(int* p, int n, int v, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
}

void launch_tables_from_state(int nn, const float4* pref, const float4* rq, const float4* tt, float4* dq, float4* cl,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_tables_from_state, dim3((nn + 255) / 256), dim3(256), 0, st, nn, pref, rq, tt, dq, cl);
}

}  // namespace swgn
