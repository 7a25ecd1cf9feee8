// Internal layout and device helpers of the swgn library (gfx950, wave64).
//
// Device-resident state of one stream, all structure-of-arrays:
//   surfels (sorted so that surfels with the same set of 4 nodes are
//   contiguous; `orig` maps back to the caller's index):
//     px,py,pz,nx,ny,nz  float[ns]    reference position and normal
//     idx                int4[ns]     4 nearest nodes, nearest first
//     w                  float4[ns]   normalised blend weights
//     orig               int[ns]
//   runs: run_start[nruns+1], maximal ranges of surfels with one node set
//   nodes:
//     pref  float4[nn]   reference position p_j
//     rq    float4[nn]   rotation quaternion (w,x,y,z), w >= 0
//     tt    float4[nn]   translation
//     dq    float4[2nn]  dual quaternion (r_j, d_j), d = 1/2 (0,t) r
//     cl    float4[nn]   live node position c_j = T_j p_j
//     nbr   int[8nn]     8 nearest other nodes
//   J^T J in block-sparse form: upper blocks (row <= col), 6x6 row-major fp32
//     row_ptr[nn+1], col_idx[nb], blk_row[nb]   (diagonal first in each row)
//     ent_ptr[nb+1], ent[ne]   per block: (run << 4 | pos_a << 2 | pos_b), the
//                              runs whose node set holds both block nodes
//     frow_ptr[nn+1], fblk[nf] full symmetric rows for the product: block id,
//                              bit 31 set when the block is used transposed
//   per frame: depth float[npx], nmap float4[npx] (normal, depth; depth 0 =
//   no normal), zbuf u64[npx]; per iteration: J float[24][pitch] (node
//   positions in ascending node order x 6), res float[pitch].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swgn {

// ---------------------------------------------------------------------------
// Global-memory accesses through a descriptor's pointers. Those pointers are
// generic, so a plain access compiles to a flat instruction, which counts
// against the LDS counter as well: every later LDS access or cross-lane
// shuffle (ds_bpermute) would then wait for the memory access to complete.
// These compile to global instructions, which only the memory counter tracks.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T gld(const T* p) {
    typedef __attribute__((address_space(1))) const T GT;
    return *(GT*)(p);
}
// (HIP's vector types cannot be copied out of another address space: a
// float2 is loaded as one 64-bit word)
__device__ __forceinline__ float2 gld2(const float2* p) {
    typedef __attribute__((address_space(1))) const unsigned long long GU;
    const unsigned long long w = *(GU*)(p);
    return make_float2(__uint_as_float((unsigned)w), __uint_as_float((unsigned)(w >> 32)));
}
template <class T>
__device__ __forceinline__ void gst(T* p, T v) {
    typedef __attribute__((address_space(1))) T GT;
    *(GT*)(p) = v;
}
typedef float f32x4n __attribute__((ext_vector_type(4)));
typedef int i32x4n __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 gld4(const float4* p) {
    typedef __attribute__((address_space(1))) const f32x4n G;
    const f32x4n v = *(G*)(p);
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ int4 gld4(const int4* p) {
    typedef __attribute__((address_space(1))) const i32x4n G;
    const i32x4n v = *(G*)(p);
    return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gst4(float4* p, float4 v) {
    typedef __attribute__((address_space(1))) f32x4n G;
    f32x4n w;
    w.x = v.x; w.y = v.y; w.z = v.z; w.w = v.w;
    *(G*)(p) = w;
}


constexpr int kWave = 64;
constexpr uint32_t kTransposed = 0x80000000u;
constexpr float kBlendEps = 1e-12f;

// --- quaternion helpers (w, x, y, z) in float4 as (x=w, y=x, z=y, w=z) -----
// A quaternion q is stored as float4{q.w, q.x, q.y, q.z} in fields .x .y .z .w
struct Q4 {
    float w, x, y, z;
};

__device__ __forceinline__ Q4 q4(float4 v) { return Q4{v.x, v.y, v.z, v.w}; }
__device__ __forceinline__ float4 f4(Q4 q) { return make_float4(q.w, q.x, q.y, q.z); }

__device__ __forceinline__ Q4 qmul(Q4 a, Q4 b) {
    Q4 r;
    r.w = ((a.w * b.w - a.x * b.x) - a.y * b.y) - a.z * b.z;
    r.x = ((a.w * b.x + a.x * b.w) + a.y * b.z) - a.z * b.y;
    r.y = ((a.w * b.y - a.x * b.z) + a.y * b.w) + a.z * b.x;
    r.z = ((a.w * b.z + a.x * b.y) - a.y * b.x) + a.z * b.w;
    return r;
}

// vector part of x (x) conj(y)
__device__ __forceinline__ float3 vec_mul_conj(Q4 x, Q4 y) {
    float3 r;
    r.x = (y.w * x.x - x.w * y.x) - (x.y * y.z - x.z * y.y);
    r.y = (y.w * x.y - x.w * y.y) - (x.z * y.x - x.x * y.z);
    r.z = (y.w * x.z - x.w * y.z) - (x.x * y.y - x.y * y.x);
    return r;
}

__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float dot3(float3 a, float3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ __forceinline__ float3 add3(float3 a, float3 b) { return make_float3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float3 sub3(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 scale3(float3 a, float s) { return make_float3(a.x * s, a.y * s, a.z * s); }

// Rotate v by unit quaternion (c0, u): v + 2 c0 (u x v) + 2 u x (u x v).
__device__ __forceinline__ float3 qrot(float c0, float3 u, float3 v) {
    float3 uv = cross3(u, v);
    float3 uuv = cross3(u, uv);
    return add3(add3(v, scale3(uv, 2.0f * c0)), scale3(uuv, 2.0f));
}

// Insert (key, j) into the ascending K-nearest list (kd, ki); equal keys keep
// the earlier (lower) index first, so scanning j upwards breaks ties to the
// lower index.
template <int K>
__device__ __forceinline__ void knn_insert(float (&kd)[K], int (&ki)[K], float key, int j) {
    if (!(key < kd[K - 1])) return;
    int p = K - 1;
#pragma unroll
    for (int q = K - 1; q > 0; --q) {
        if (key < kd[q - 1]) {
            kd[q] = kd[q - 1];
            ki[q] = ki[q - 1];
            p = q - 1;
        }
    }
    kd[p] = key;
    ki[p] = j;
}

// Insert (key, j) into the K-nearest list ascending in (key, j), whatever the
// order the candidates come in.
template <int K>
__device__ __forceinline__ void knn_insert_lex(float (&kd)[K], int (&ki)[K], float key, int j) {
    if (!(key < kd[K - 1] || (key == kd[K - 1] && j < ki[K - 1]))) return;
    int p = K - 1;
#pragma unroll
    for (int q = K - 1; q > 0; --q) {
        if (key < kd[q - 1] || (key == kd[q - 1] && j < ki[q - 1])) {
            kd[q] = kd[q - 1];
            ki[q] = ki[q - 1];
            p = q - 1;
        }
    }
    kd[p] = key;
    ki[p] = j;
}

// Result of warping one surfel by the blend of its 4 nodes.
struct Warp {
    Q4 cr, cd;        // normalised blend c = b / |b_r|
    float inv_beta;   // 1 / |b_r|
    float sgn[4];     // hemisphere signs s_k
    float3 v, n;      // live position and normal
    bool ok;          // |b_r|^2 >= 1e-12
};

// Dual-quaternion blend (hemisphere of the nearest node) and application:
// c = b / |b_r|, v' = rot(c_r) v + 2 vec(c_d c_r*), n' = rot(c_r) n.
// Every value feeding an integer decision goes through this one function.
__device__ __forceinline__ Warp warp_surfel(int4 idx, float4 w, float3 v, float3 n,
                                            const float4* __restrict__ dq) {
    Warp out;
    const int id[4] = {idx.x, idx.y, idx.z, idx.w};
    const float wk[4] = {w.x, w.y, w.z, w.w};
    Q4 r0 = q4(gld4(dq + 2 * id[0]));
    Q4 br = {0.f, 0.f, 0.f, 0.f}, bd = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        Q4 rk = q4(gld4(dq + 2 * id[k]));
        Q4 dk = q4(gld4(dq + 2 * id[k] + 1));
        float dt = ((r0.w * rk.w + r0.x * rk.x) + r0.y * rk.y) + r0.z * rk.z;
        float s = dt >= 0.f ? 1.f : -1.f;
        out.sgn[k] = s;
        float a = wk[k] * s;
        br.w += a * rk.w; br.x += a * rk.x; br.y += a * rk.y; br.z += a * rk.z;
        bd.w += a * dk.w; bd.x += a * dk.x; bd.y += a * dk.y; bd.z += a * dk.z;
    }
    float br2 = ((br.w * br.w + br.x * br.x) + br.y * br.y) + br.z * br.z;
    out.ok = br2 >= kBlendEps;
    float ib = 1.0f / sqrtf(out.ok ? br2 : 1.0f);
    out.inv_beta = ib;
    out.cr = Q4{br.w * ib, br.x * ib, br.y * ib, br.z * ib};
    out.cd = Q4{bd.w * ib, bd.x * ib, bd.y * ib, bd.z * ib};
    float3 u = make_float3(out.cr.x, out.cr.y, out.cr.z);
    float3 t = vec_mul_conj(out.cd, out.cr);
    out.v = add3(qrot(out.cr.w, u, v), scale3(t, 2.0f));
    out.n = qrot(out.cr.w, u, n);
    return out;
}

// Camera intrinsics and gates as passed to kernels.
struct Cam {
    int W, H;
    float fx, fy, cx, cy;
};

// Pixel of a live point: floor(fx*(x/z) + cx + 0.5), inside the image, z > 0.
__device__ __forceinline__ bool project(const Cam& c, float3 v, int& ux, int& uy) {
    float px = c.fx * (v.x / v.z) + c.cx;
    float py = c.fy * (v.y / v.z) + c.cy;
    float hx = px + 0.5f;
    float hy = py + 0.5f;
    bool in = (v.z > 0.f) && (hx >= 0.f) && (hx < (float)c.W) && (hy >= 0.f) && (hy < (float)c.H);
    ux = in ? (int)floorf(hx) : 0;
    uy = in ? (int)floorf(hy) : 0;
    return in;
}

// Back-projection ((u - cx)/fx * d, (v - cy)/fy * d, d).
__device__ __forceinline__ float3 backproject(const Cam& c, int ux, int uy, float d) {
    return make_float3((((float)ux - c.cx) / c.fx) * d, (((float)uy - c.cy) / c.fy) * d, d);
}

__device__ __forceinline__ bool depth_ok(float d) { return (d > 0.f) && (d < INFINITY); }

// Node dual quaternion (r, d = 1/2 (0,t) r) and live position c = R p + t.
__device__ __forceinline__ void node_tables(float4 p, Q4 r, float3 t, float4* dq, float4* cl, int k) {
    float3 u = make_float3(r.x, r.y, r.z);
    float3 c = add3(qrot(r.w, u, make_float3(p.x, p.y, p.z)), t);
    Q4 d = qmul(Q4{0.f, t.x, t.y, t.z}, r);
    gst4(dq + 2 * k, f4(r));
    gst4(dq + 2 * k + 1, make_float4(0.5f * d.w, 0.5f * d.x, 0.5f * d.y, 0.5f * d.z));
    gst4(cl + k, make_float4(c.x, c.y, c.z, 0.f));
}

// Per Gauss-Newton iteration statistics written by the device.
struct IterStats {
    double e_data, e_reg, pcg_resid;
    int n_corr, pad;
};

// ---------------------------------------------------------------------------
// Lane exchanges on the VALU (DPP and the gfx950 permlane swaps) instead of
// the LDS crossbar (ds_bpermute): no LDS instruction, no wait on the LDS
// counter, a few cycles of latency. They move values only, so a sum built
// from them equals, bit for bit, the same sum built from __shfl_xor.
//   xchg<M>(v)    the value of lane (lane ^ M), M in {1, 2, 4, 8, 16, 32};
//                 M >= 16 needs every lane of the wave active, M <= 8 every
//                 lane of the lane's 16-lane row
//   bcast8(v, c)  the value of lane c of the lane's 8-lane group, c in [0, 8)
//                 a compile-time constant once unrolled; needs the group's
//                 lanes active
// DPP controls (gfx9): quad_perm [a,b,c,d] = a | b << 2 | c << 4 | d << 6,
// row_shl:n = 0x100 + n (lane i takes lane i + n of its 16-lane row),
// row_shr:n = 0x110 + n (lane i takes lane i - n), row_ror:n = 0x120 + n;
// a bank is 4 lanes of a row, and lanes of banks left out of the bank mask
// keep the first operand.
// ---------------------------------------------------------------------------
template <int CTRL, int BANKS = 0xF>
__device__ __forceinline__ int dpp_mov(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, CTRL, 0xF, BANKS, false);
}

template <int M>
__device__ __forceinline__ int xchg_i(int v) {
    static_assert(M == 1 || M == 2 || M == 4 || M == 8 || M == 16 || M == 32, "xor mask");
    if constexpr (M == 1) {
        return dpp_mov<0xB1>(0, v);                     // quad_perm [1,0,3,2]
    } else if constexpr (M == 2) {
        return dpp_mov<0x4E>(0, v);                     // quad_perm [2,3,0,1]
    } else if constexpr (M == 4) {
        const int t = dpp_mov<0x104, 0x5>(v, v);        // banks 0, 2: lane + 4
        return dpp_mov<0x114, 0xA>(t, v);               // banks 1, 3: lane - 4
    } else if constexpr (M == 8) {
        return dpp_mov<0x128>(0, v);                    // row_ror:8
    } else if constexpr (M == 16) {
        // odd rows of the first operand trade places with even rows of the second
        const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (threadIdx.x & 16) ? (int)p[0] : (int)p[1];
    } else {
        // rows 2, 3 of the first operand trade places with rows 0, 1 of the second
        const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (threadIdx.x & 32) ? (int)p[0] : (int)p[1];
    }
}

template <int M>
__device__ __forceinline__ float xchg(float v) {
    return __int_as_float(xchg_i<M>(__float_as_int(v)));
}
template <int M>
__device__ __forceinline__ double xchg(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)xchg_i<M>((int)(unsigned)b);
    const unsigned hi = (unsigned)xchg_i<M>((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int C>
__device__ __forceinline__ int bcast8_i(int v) {
    if constexpr (C < 4) {
        const int q = dpp_mov<C * 0x55>(0, v);          // lane C of each quad
        return dpp_mov<0x114, 0xA>(q, q);               // the group's upper quad from its lower
    } else {
        const int q = dpp_mov<(C - 4) * 0x55>(0, v);
        return dpp_mov<0x104, 0x5>(q, q);               // the group's lower quad from its upper
    }
}
__device__ __forceinline__ int bcast8_i(int v, int c) {
    switch (c) {
        case 0: return bcast8_i<0>(v);
        case 1: return bcast8_i<1>(v);
        case 2: return bcast8_i<2>(v);
        case 3: return bcast8_i<3>(v);
        case 4: return bcast8_i<4>(v);
        case 5: return bcast8_i<5>(v);
        case 6: return bcast8_i<6>(v);
        default: return bcast8_i<7>(v);
    }
}
__device__ __forceinline__ float bcast8(float v, int c) { return __int_as_float(bcast8_i(__float_as_int(v), c)); }
__device__ __forceinline__ double bcast8(double v, int c) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)bcast8_i((int)(unsigned)b, c);
    const unsigned hi = (unsigned)bcast8_i((int)(unsigned)(b >> 32), c);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// ---------------------------------------------------------------------------
// Wave and block reductions (fixed butterfly order)
// ---------------------------------------------------------------------------
// Sums over the wave in the butterfly order 32, 16, 8, 4, 2, 1 through the
// lane exchanges above (every lane active; every lane ends with the same
// value, the one a __shfl_xor butterfly gives).
template <class T>
__device__ __forceinline__ T wave_sum_t(T v) {
    v += xchg<32>(v);
    v += xchg<16>(v);
    v += xchg<8>(v);
    v += xchg<4>(v);
    v += xchg<2>(v);
    v += xchg<1>(v);
    return v;
}
__device__ __forceinline__ double wave_sum(double v) { return wave_sum_t(v); }
__device__ __forceinline__ float wave_sumf(float v) { return wave_sum_t(v); }
__device__ __forceinline__ int wave_sumi(int v) {
    v += xchg_i<32>(v);
    v += xchg_i<16>(v);
    v += xchg_i<8>(v);
    v += xchg_i<4>(v);
    v += xchg_i<2>(v);
    v += xchg_i<1>(v);
    return v;
}

// Block sum over blockDim.x (multiple of 64, <= 1024) threads; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    if (l == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        int nw = blockDim.x / kWave;
        for (int q = 0; q < nw; ++q) t += sh[q];
    }
    __syncthreads();
    return t;
}


// Cross-lane sums with DPP (gfx9): every lane of a 16-lane row ends with the
// row's sum after mirror, half-mirror and two quad permutations. The order of
// additions is fixed per lane, so results are reproducible.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float row16_sum(float v) {
    v += dpp<0x140>(v);   // row_mirror
    v += dpp<0x141>(v);   // row_half_mirror
    v += dpp<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);    // quad_perm [2,3,0,1]
    return v;
}
__device__ __forceinline__ float readlane_f(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
// Sum over the whole wave (all lanes active), uniform result.
__device__ __forceinline__ float wave64_sum(float v) {
    v = row16_sum(v);
    return (readlane_f(v, 0) + readlane_f(v, 16)) + (readlane_f(v, 32) + readlane_f(v, 48));
}

}  // namespace swgn
