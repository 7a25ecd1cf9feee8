// Depth-map fusion into the live surfels (Sec. 5, Sec. 6.1) and the return of
// fused surfels to the reference frame (Sec. 6.4), for one stream.
//
//   fuse_live    warp every surfel by the current field (live position and
//                normal kept for the match), and its point into an index map
//                super-sampled 4x4 over the depth map: 64-bit atomicMin of
//                (z bits << 32 | caller index), nearest z, then lower index
//   fuse_match   one thread per depth pixel with a normal: the 16 sub-pixels
//                of its 4x4 block are the candidates; a candidate passes if
//                |v - V(u)|^2 <= delta_d^2 and n . N(u) >= delta_n (FP32, one
//                operation order); of those the highest confidence wins, then
//                the smaller squared distance, then the lower caller index.
//                The depth surfel (V, N, confidence exp(-gamma^2 / (2 phi^2)),
//                radius sqrt(2) d / (fx max(|n_z|, cos 75 deg))) is fused into
//                the winner: c += c_d, t = t_now, v, n, r confidence-weighted
//                (n renormalised); the fused live surfel goes back to the
//                reference frame through the inverse of its own blend. A
//                surfel lies in exactly one pixel's block, so no two threads
//                fuse into the same surfel.
#include "swgn_fusion.h"
#include "swgn_impl.h"

namespace swgn {

namespace {

__device__ __forceinline__ unsigned long long fuse_key(float z, int orig) {
    return ((unsigned long long)__float_as_uint(z) << 32) | (unsigned long long)(unsigned)orig;
}

// Super-sampled pixel (floor(4 hx), floor(4 hy)), hx = fx (x / z) + cx + 1/2:
// the depth pixel's own rule scaled by 4 (exact in FP32), so the sub-pixel
// lies in the point's depth pixel.
__device__ __forceinline__ bool subpixel(const Cam& c, float3 v, int& sx, int& sy) {
    const float hx = (c.fx * (v.x / v.z) + c.cx) + 0.5f;
    const float hy = (c.fy * (v.y / v.z) + c.cy) + 0.5f;
    const bool in = (v.z > 0.f) && (hx >= 0.f) && (hx < (float)c.W) && (hy >= 0.f) && (hy < (float)c.H);
    sx = in ? (int)floorf(4.0f * hx) : 0;
    sy = in ? (int)floorf(4.0f * hy) : 0;
    return in;
}

__global__ void __launch_bounds__(256) k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(256) k_fuse_live(FuseArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.ns) return;
    const float3 v = make_float3(a.px[i], a.py[i], a.pz[i]);
    const float3 n = make_float3(a.nx[i], a.ny[i], a.nz[i]);
    const Warp wp = warp_surfel(a.idx[i], a.w[i], v, n, a.dq);
    const float nanv = __int_as_float(0x7fc00000);
    a.lx[i] = wp.ok ? wp.v.x : nanv;
    a.ly[i] = wp.ok ? wp.v.y : nanv;
    a.lz[i] = wp.ok ? wp.v.z : nanv;
    a.lnx[i] = wp.n.x;
    a.lny[i] = wp.n.y;
    a.lnz[i] = wp.n.z;
    int sx, sy;
    if (wp.ok && subpixel(a.cam, wp.v, sx, sy))
        atomicMin(&a.zmap4[(int64_t)sy * (4 * a.cam.W) + sx], fuse_key(wp.v.z, a.orig[i]));
}

__global__ void __launch_bounds__(256) k_fuse_match(FuseArgs a) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int npx = a.cam.W * a.cam.H;
    const bool in = u < npx;
    const int x = in ? u % a.cam.W : 0, y = in ? u / a.cam.W : 0;
    const float4 nm = in ? a.nmap[u] : make_float4(0.f, 0.f, 0.f, 0.f);
    int best = -1, best_orig = 0x7fffffff;
    float best_c = 0.f, best_d2 = 0.f;
    const float d = nm.w;
    const float3 V = make_float3((((float)x - a.cam.cx) / a.cam.fx) * d, (((float)y - a.cam.cy) / a.cam.fy) * d, d);
    if (nm.w > 0.f) {
        // the 16 keys, then the occupied ones' sorted indices, then their live
        // surfels: three rounds of independent loads instead of a chain per
        // candidate (the winner does not depend on the visiting order)
        const int W4 = 4 * a.cam.W;
        unsigned long long key[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) key[q] = a.zmap4[(int64_t)(4 * y + (q >> 2)) * W4 + 4 * x + (q & 3)];
        int sid[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) sid[q] = key[q] != ~0ull ? a.inv[(int)(unsigned)(key[q] & 0xffffffffu)] : -1;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int s = sid[q];
            if (s < 0) continue;
            const int org = (int)(unsigned)(key[q] & 0xffffffffu);
            const float dx = a.lx[s] - V.x, dy = a.ly[s] - V.y, dz = a.lz[s] - V.z;
            const float d2 = (dx * dx + dy * dy) + dz * dz;
            const float dot = (a.lnx[s] * nm.x + a.lny[s] * nm.y) + a.lnz[s] * nm.z;
            const float c = a.conf[s];
            if (!(d2 <= a.dist2) || !(dot >= a.cosn)) continue;
            const bool better = best < 0 || c > best_c || (c == best_c && (d2 < best_d2 ||
                                                                     (d2 == best_d2 && org < best_orig)));
            if (better) {
                best = s;
                best_orig = org;
                best_c = c;
                best_d2 = d2;
            }
        }
    }
    // counts summed per wave, one atomic each: fused pixels and append
    // candidates (pixels with a normal and no surfel, Sec. 6.4)
    const unsigned long long bf = __ballot(best >= 0), bc = __ballot(nm.w > 0.f && best < 0);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (bf) atomicAdd(&a.counts[0], __popcll(bf));
        if (bc) atomicAdd(&a.counts[1], __popcll(bc));
    }
    if (!in) return;
    a.match[u] = best < 0 ? -1 : best_orig;
    if (best < 0) return;
    // the depth surfel (Sec. 5)
    const float gx = (float)x - a.cam.cx, gy = (float)y - a.cam.cy;
    const float gamma2 = (gx * gx + gy * gy) / (a.cam.cx * a.cam.cx + a.cam.cy * a.cam.cy);
    const float cd = expf(-gamma2 / (2.0f * kFusePhi * kFusePhi));
    const float rd = 1.41421356237f * d / (a.cam.fx * fmaxf(fabsf(nm.z), a.cos_max));
    // fusion (Sec. 6.1)
    const int s = best;
    const float c0 = a.conf[s], c1 = c0 + cd;
    const float3 lv = make_float3(a.lx[s], a.ly[s], a.lz[s]);
    const float3 ln = make_float3(a.lnx[s], a.lny[s], a.lnz[s]);
    const float3 v1 = make_float3((c0 * lv.x + cd * V.x) / c1, (c0 * lv.y + cd * V.y) / c1, (c0 * lv.z + cd * V.z) / c1);
    float3 n1 = make_float3((c0 * ln.x + cd * nm.x) / c1, (c0 * ln.y + cd * nm.y) / c1, (c0 * ln.z + cd * nm.z) / c1);
    const float il = 1.0f / sqrtf((n1.x * n1.x + n1.y * n1.y) + n1.z * n1.z);
    n1 = make_float3(n1.x * il, n1.y * il, n1.z * il);
    a.radius[s] = (c0 * a.radius[s] + cd * rd) / c1;
    a.conf[s] = c1;
    a.t_obs[s] = a.t_now;
    // back to the reference frame (Sec. 6.4): the inverse of the surfel's own
    // normalised blend, v = R^T (v' - t), n = R^T n'
    const float3 v0 = make_float3(a.px[s], a.py[s], a.pz[s]);
    const float3 n0 = make_float3(a.nx[s], a.ny[s], a.nz[s]);
    const Warp wp = warp_surfel(a.idx[s], a.w[s], v0, n0, a.dq);
    const float3 u3 = make_float3(-wp.cr.x, -wp.cr.y, -wp.cr.z);     // conjugate rotation
    const float3 tb = scale3(vec_mul_conj(wp.cd, wp.cr), 2.0f);
    const float3 vr = qrot(wp.cr.w, u3, sub3(v1, tb));
    const float3 nr = qrot(wp.cr.w, u3, n1);
    a.px[s] = vr.x; a.py[s] = vr.y; a.pz[s] = vr.z;
    a.nx[s] = nr.x; a.ny[s] = nr.y; a.nz[s] = nr.z;
    const int o = best_orig;
    a.cpos[3 * o + 0] = vr.x; a.cpos[3 * o + 1] = vr.y; a.cpos[3 * o + 2] = vr.z;
    a.cnrm[3 * o + 0] = nr.x; a.cnrm[3 * o + 1] = nr.y; a.cnrm[3 * o + 2] = nr.z;
    a.crad[o] = a.radius[s];
    a.cconf[o] = c1;
    a.ctobs[o] = a.t_now;
}

__global__ void __launch_bounds__(256) k_fuse_gather(int ns, const int* __restrict__ orig,
        const float* __restrict__ crad, const float* __restrict__ cconf, const int* __restrict__ ctobs,
        float* __restrict__ rad, float* __restrict__ conf, int* __restrict__ tobs, int* __restrict__ inv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns) return;
    const int o = orig[i];
    rad[i] = crad[o];
    conf[i] = cconf[o];
    tobs[i] = ctobs[o];
    inv[o] = i;
}

}  // namespace

void launch_fuse_gather(int ns, const int* orig, const float* crad, const float* cconf, const int* ctobs,
                        float* rad, float* conf, int* tobs, int* inv, hipStream_t st) {
    if (ns > 0)
        hipLaunchKernelGGL(k_fuse_gather, dim3((ns + 255) / 256), dim3(256), 0, st, ns, orig, crad, cconf, ctobs,
                           rad, conf, tobs, inv);
}

void launch_fuse(const FuseArgs& a, hipStream_t st) {
    const int64_t n4 = (int64_t)16 * a.cam.W * a.cam.H;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, st, a.zmap4, n4, ~0ull);
    if (a.ns > 0) hipLaunchKernelGGL(k_fuse_live, dim3((a.ns + 255) / 256), dim3(256), 0, st, a);
    const int npx = a.cam.W * a.cam.H;
    hipLaunchKernelGGL(k_fuse_match, dim3((npx + 255) / 256), dim3(256), 0, st, a);
}

}  // namespace swgn
