// Per-frame kernels of the Gauss-Newton warp-field solve (Sec. 7, Sec. 8).
//
//   depth_prep   normal map of the depth image (Sec. 5)
//   clear_z      index-map reset
//   warp_zbuf    dual-quaternion warp of every surfel (Sec. 3, Eq. 1-2) and
//                a 64-bit atomic-min z-buffer of (z bits, surfel index) (Sec. 7)
//   corr_jac     projective correspondence, point-to-plane residual and its
//                exact Jacobian with respect to the 4 node twists
//   assemble     J^T J and J^T r as 6x6 blocks over node pairs, with the
//                as-rigid-as-possible terms; one wave per block, no float atomics
//   jacobi       FP64 inverses of the 6x6 diagonal blocks
//   pcg_*        block-Jacobi preconditioned conjugate gradients, scalars on
//                the device
//   node_update  T_k <- Delta_k(xi_k) o T_k
//
// Sums are taken in a fixed order everywhere, so a frame solve is
// bit-reproducible run to run.
#include "swgn_impl.h"
#include "swgn_launch.h"

namespace swgn {

// ---------------------------------------------------------------------------
// Wave and block reductions (fixed butterfly order)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ float wave_sumf(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ int wave_sumi(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
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

// Sum of n partials in a fixed order by one block; result valid in all threads.
__device__ __forceinline__ double reduce_partials(const double* __restrict__ part, int n, double* sh) {
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
    double t = block_sum(v, sh);
    if (threadIdx.x == 0) sh[32] = t;
    __syncthreads();
    double r = sh[32];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// Depth preprocessing: normal map by central differences (Sec. 5).
// nmap = (n, d) where the normal is defined, (0, 0, 0, 0) elsewhere.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_depth_prep(Cam cam, const float* __restrict__ depth, float gate,
                                                    float4* __restrict__ nmap) {
    int x = blockIdx.x * 16 + (threadIdx.x & 15);
    int y = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (x >= cam.W || y >= cam.H) return;
    int W = cam.W;
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
    float* J;              // [24][pitch]
    float* res;            // [pitch]
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
        // store by node position within the surfel's ascending node set
        const int ids[4] = {id.x, id.y, id.z, id.w};
        float* J = o.J;
        int P = o.pitch;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int pos = (ids[0] < ids[k]) + (ids[1] < ids[k]) + (ids[2] < ids[k]) + (ids[3] < ids[k]);
            float* Jp = J + (size_t)(pos * 6) * P + i;
            Jp[0] = Jw[k][0];
            Jp[(size_t)P] = Jw[k][1];
            Jp[(size_t)2 * P] = Jw[k][2];
            Jp[(size_t)3 * P] = Jt[k][0];
            Jp[(size_t)4 * P] = Jt[k][1];
            Jp[(size_t)5 * P] = Jt[k][2];
        }
        o.res[i] = r;
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

// ---------------------------------------------------------------------------
// Assembly of J^T J (+ mu I) and J^T r, one wave per upper block.
// ---------------------------------------------------------------------------
struct AsmIn {
    int nb, nn, pitch;
    const int* blk_row;
    const int* col_idx;
    const int* ent_ptr;
    const uint32_t* ent;
    const int* run_start;
    const float* J;
    const float* res;
    const int* nbr;
    const float4* pref;
    const float4* rq;
    const float4* cl;
    const int* frow_ptr;
    const int* fcol;
    float lambda, mu;
};

struct AsmOut {
    float* H;       // [nb][36]
    float* g;       // [nn][6]
    float* ereg;    // [nn] sum over out-edges of |r_jm|^2
};

__device__ __forceinline__ float3 ld3(float4 a) { return make_float3(a.x, a.y, a.z); }

// y = R_m (p_j - p_m), r_jm = c_j - c_m - y
__device__ __forceinline__ void arap_edge(const AsmIn& in, int j, int m, float3& y, float3& r) {
    float3 pj = ld3(in.pref[j]), pm = ld3(in.pref[m]);
    float4 q = in.rq[m];
    y = qrot(q.x, make_float3(q.y, q.z, q.w), sub3(pj, pm));
    r = sub3(sub3(ld3(in.cl[j]), ld3(in.cl[m])), y);
}

__global__ void __launch_bounds__(256) k_assemble(AsmIn in, AsmOut out) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int b = blockIdx.x * (blockDim.x / kWave) + wave;
    if (b >= in.nb) return;
    const int k = in.blk_row[b], l = in.col_idx[b];
    const bool diag = (k == l);
    float acc[36];
    float gacc[6];
    float er = 0.f;
#pragma unroll
    for (int t = 0; t < 36; ++t) acc[t] = 0.f;
#pragma unroll
    for (int t = 0; t < 6; ++t) gacc[t] = 0.f;

    const int e0 = in.ent_ptr[b], e1 = in.ent_ptr[b + 1];
    const size_t P = (size_t)in.pitch;
    for (int eb = e0; eb < e1; eb += kWave) {
        int j = eb + lane;
        bool have = j < e1;
        uint32_t e = have ? in.ent[j] : 0u;
        int run = (int)(e >> 4);
        int st = have ? in.run_start[run] : 0;
        int len = have ? in.run_start[run + 1] - st : 0;
        int pp = (int)(e & 15u);
        int incl = len;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            int t = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += t;
        }
        int total = __shfl(incl, kWave - 1, kWave);
        for (int f0 = 0; f0 < total; f0 += kWave) {
            int f = f0 + lane;
            int lo = 0, hi = kWave - 1;
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                int mid = (lo + hi) >> 1;
                int v = __shfl(incl, mid, kWave);
                if (v > f) hi = mid; else lo = mid + 1;
            }
            int inc_j = __shfl(incl, lo, kWave);
            int len_j = __shfl(len, lo, kWave);
            int st_j = __shfl(st, lo, kWave);
            int pp_j = __shfl(pp, lo, kWave);
            if (f < total) {
                int sidx = st_j + (f - (inc_j - len_j));
                int pa = pp_j >> 2, pb = pp_j & 3;
                const float* Ja = in.J + (size_t)(pa * 6) * P + sidx;
                float xa[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) xa[c] = Ja[c * P];
                if (diag) {
                    float rr = in.res[sidx];
#pragma unroll
                    for (int a = 0; a < 6; ++a) {
#pragma unroll
                        for (int c = a; c < 6; ++c) acc[a * 6 + c] = fmaf(xa[a], xa[c], acc[a * 6 + c]);
                        gacc[a] = fmaf(xa[a], rr, gacc[a]);
                    }
                } else {
                    const float* Jb = in.J + (size_t)(pb * 6) * P + sidx;
                    float xb[6];
#pragma unroll
                    for (int c = 0; c < 6; ++c) xb[c] = Jb[c * P];
#pragma unroll
                    for (int a = 0; a < 6; ++a)
#pragma unroll
                        for (int c = 0; c < 6; ++c) acc[a * 6 + c] = fmaf(xa[a], xb[c], acc[a * 6 + c]);
                }
            }
        }
    }

    // as-rigid-as-possible terms, weight lambda
    const float lam = in.lambda;
    if (diag) {
        if (lane < 8) {                       // out-edge k -> m: J_k = [0 | I]
            int m = in.nbr[8 * k + lane];
            float3 y, r;
            arap_edge(in, k, m, y, r);
            acc[21] += lam; acc[28] += lam; acc[35] += lam;
            gacc[3] += lam * r.x; gacc[4] += lam * r.y; gacc[5] += lam * r.z;
            er += dot3(r, r);
        }
        // in-edges j -> k: J_k = [[y]x | -I]
        const int f0 = in.frow_ptr[k], f1 = in.frow_ptr[k + 1];
        for (int f = f0 + lane; f < f1; f += kWave) {
            int j = in.fcol[f];
            if (j == k) continue;
            bool edge = false;
#pragma unroll
            for (int q = 0; q < 8; ++q) edge |= (in.nbr[8 * j + q] == k);
            if (!edge) continue;
            float3 y, r;
            arap_edge(in, j, k, y, r);
            float yy = dot3(y, y);
            // [[|y|^2 I - y y^T, [y]x], [-[y]x, I]] (upper triangle)
            acc[0] += lam * (yy - y.x * y.x); acc[1] += lam * (-y.x * y.y); acc[2] += lam * (-y.x * y.z);
            acc[7] += lam * (yy - y.y * y.y); acc[8] += lam * (-y.y * y.z);
            acc[14] += lam * (yy - y.z * y.z);
            // [y]x = [[0,-yz,yy],[yz,0,-yx],[-yy,yx,0]]
            acc[4] += lam * (-y.z); acc[5] += lam * (y.y);
            acc[9] += lam * (y.z);  acc[11] += lam * (-y.x);
            acc[15] += lam * (-y.y); acc[16] += lam * (y.x);
            acc[21] += lam; acc[28] += lam; acc[35] += lam;
            // g += lambda [r x y; -r]
            float3 rxy = cross3(r, y);
            gacc[0] += lam * rxy.x; gacc[1] += lam * rxy.y; gacc[2] += lam * rxy.z;
            gacc[3] -= lam * r.x; gacc[4] -= lam * r.y; gacc[5] -= lam * r.z;
        }
    } else {
        if (lane == 0) {
            bool e_kl = false;
#pragma unroll
            for (int q = 0; q < 8; ++q) e_kl |= (in.nbr[8 * k + q] == l);
            if (e_kl) {                       // edge k -> l: J_k^T J_l = [0 0; [y]x -I]
                float3 y, r;
                arap_edge(in, k, l, y, r);
                acc[19] += lam * (-y.z); acc[20] += lam * (y.y);
                acc[24] += lam * (y.z);  acc[26] += lam * (-y.x);
                acc[30] += lam * (-y.y); acc[31] += lam * (y.x);
                acc[21] -= lam; acc[28] -= lam; acc[35] -= lam;
            }
        } else if (lane == 1) {
            bool e_lk = false;
#pragma unroll
            for (int q = 0; q < 8; ++q) e_lk |= (in.nbr[8 * l + q] == k);
            if (e_lk) {                       // edge l -> k: J_k^T J_l = [0 -[y]x; 0 -I]
                float3 y, r;
                arap_edge(in, l, k, y, r);
                acc[4] += lam * (y.z);  acc[5] += lam * (-y.y);
                acc[9] += lam * (-y.z); acc[11] += lam * (y.x);
                acc[15] += lam * (y.y); acc[16] += lam * (-y.x);
                acc[21] -= lam; acc[28] -= lam; acc[35] -= lam;
            }
        }
    }

#pragma unroll
    for (int t = 0; t < 36; ++t) acc[t] = wave_sumf(acc[t]);
#pragma unroll
    for (int t = 0; t < 6; ++t) gacc[t] = wave_sumf(gacc[t]);
    er = wave_sumf(er);

    float* Hb = out.H + (size_t)b * 36;
    if (diag) {
        if (lane < 36) {
            int a = lane / 6, c = lane % 6;
            float v = 0.f;
#pragma unroll
            for (int t = 0; t < 36; ++t) {
                int ta = t / 6, tc = t % 6;
                if ((ta == min(a, c)) && (tc == max(a, c))) v = acc[t];
            }
            if (a == c) v += in.mu;
            Hb[lane] = v;
        }
        if (lane < 6) {
            float v = 0.f;
#pragma unroll
            for (int t = 0; t < 6; ++t) if (t == lane) v = gacc[t];
            out.g[6 * k + lane] = v;
        }
        if (lane == 0) out.ereg[k] = er;
    } else {
        if (lane < 36) {
            float v = 0.f;
#pragma unroll
            for (int t = 0; t < 36; ++t) if (t == lane) v = acc[t];
            Hb[lane] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// Block-Jacobi inverses (FP64) + per-iteration energy statistics
// ---------------------------------------------------------------------------
struct IterStats {
    double e_data, e_reg, pcg_resid;
    int n_corr, pad;
};

__global__ void __launch_bounds__(256) k_jacobi(int nn, const int* __restrict__ row_ptr,
        const float* __restrict__ H, double* __restrict__ Minv, int* __restrict__ flags,
        const double* __restrict__ part_e, const int* __restrict__ part_n, int nparts,
        const float* __restrict__ ereg, IterStats* __restrict__ stats) {
    __shared__ double sh[40];
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nn) {
        const float* A = H + (size_t)row_ptr[k] * 36;
        double L[6][6];
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 6; ++a)
#pragma unroll
            for (int c = 0; c < 6; ++c) L[a][c] = 0.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            double d = (double)A[c * 6 + c];
            for (int t = 0; t < c; ++t) d -= L[c][t] * L[c][t];
            ok = ok && (d > 0.0);
            double lc = sqrt(ok ? d : 1.0);
            L[c][c] = lc;
            for (int a = c + 1; a < 6; ++a) {
                double v = (double)A[c * 6 + a];
                for (int t = 0; t < c; ++t) v -= L[a][t] * L[c][t];
                L[a][c] = v / lc;
            }
        }
        double* M = Minv + (size_t)k * 36;
        if (!ok) {
            atomicOr(flags, 1);
            for (int t = 0; t < 36; ++t) M[t] = (t % 7 == 0) ? 1.0 : 0.0;
        } else {
            // inverse of L (lower), then M = L^-T L^-1
            double Li[6][6];
#pragma unroll
            for (int a = 0; a < 6; ++a)
#pragma unroll
                for (int c = 0; c < 6; ++c) Li[a][c] = 0.0;
            for (int c = 0; c < 6; ++c) {
                Li[c][c] = 1.0 / L[c][c];
                for (int a = c + 1; a < 6; ++a) {
                    double v = 0.0;
                    for (int t = c; t < a; ++t) v -= L[a][t] * Li[t][c];
                    Li[a][c] = v / L[a][a];
                }
            }
            for (int a = 0; a < 6; ++a)
                for (int c = 0; c < 6; ++c) {
                    double v = 0.0;
                    for (int t = max(a, c); t < 6; ++t) v += Li[t][a] * Li[t][c];
                    M[a * 6 + c] = v;
                }
        }
    }
    if (blockIdx.x == 0) {
        double e = 0.0;
        for (int q = threadIdx.x; q < nparts; q += blockDim.x) e += part_e[q];
        e = block_sum(e, sh);
        double n = 0.0;
        for (int q = threadIdx.x; q < nparts; q += blockDim.x) n += (double)part_n[q];
        n = block_sum(n, sh);
        double er = 0.0;
        for (int q = threadIdx.x; q < nn; q += blockDim.x) er += (double)ereg[q];
        er = block_sum(er, sh);
        if (threadIdx.x == 0) {
            stats->e_data = e;
            stats->e_reg = er;
            stats->n_corr = (int)n;
            if (!(e < INFINITY) || !(er < INFINITY)) atomicOr(flags, 2);
        }
    }
}

// ---------------------------------------------------------------------------
// Block-Jacobi PCG on (J^T J + mu I) delta = -g.
//   scalars sc[2 it] = rho_it, sc[2 it + 1] = p_it . q_it
// ---------------------------------------------------------------------------
struct PcgVec {
    float *x, *r, *z, *q;
    float* p[2];              // ping-pong search directions
    const double* Minv;
    double* sc;
    double* part_rho;         // per update block
    double* part_rr;
    double* part_pq;          // per spmv block
    int n_upd_blocks, n_spmv_blocks;
};

__device__ __forceinline__ void apply_minv(const double* __restrict__ M, const float* r, double* z) {
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        double v = 0.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) v += M[a * 6 + c] * (double)r[c];
        z[a] = v;
    }
}

__global__ void __launch_bounds__(256) k_pcg_init(int nn, const float* __restrict__ g, PcgVec v) {
    __shared__ double sh[40];
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    double rho = 0.0, rr = 0.0;
    if (k < nn) {
        float r[6];
        double z[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) r[c] = -g[6 * k + c];
        apply_minv(v.Minv + (size_t)k * 36, r, z);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            float zf = (float)z[c];
            v.r[6 * k + c] = r[c];
            v.z[6 * k + c] = zf;
            v.p[0][6 * k + c] = zf;
            v.x[6 * k + c] = 0.f;
            rho += (double)r[c] * (double)zf;
            rr += (double)r[c] * (double)r[c];
        }
    }
    rho = block_sum(rho, sh);
    rr = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        v.part_rho[blockIdx.x] = rho;
        v.part_rr[blockIdx.x] = rr;
    }
}

// q = A p_it for one (row node, component) per thread; p_it = z + beta p_{it-1}
// is formed on the fly for it > 0.
__global__ void __launch_bounds__(256) k_pcg_spmv(int nn, int it, const int* __restrict__ frow_ptr,
        const uint32_t* __restrict__ fblk, const int* __restrict__ fcol, const float* __restrict__ H, PcgVec v) {
    __shared__ double sh[40];
    double rho = reduce_partials(v.part_rho, v.n_upd_blocks, sh);
    bool stop = (rho == 0.0);
    double beta = 0.0;
    if (it > 0 && !stop) beta = rho / v.sc[2 * (it - 1)];
    if (blockIdx.x == 0 && threadIdx.x == 0) v.sc[2 * it] = rho;
    const float bf = (float)beta;
    // p_it lives in p[it & 1]; p_0 was written by the init kernel
    const float* pold = it > 0 ? v.p[(it + 1) & 1] : v.p[0];
    float* pnew = v.p[it & 1];
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    double pq = 0.0;
    if (!stop && t < 6 * nn) {
        int k = t / 6, a = t % 6;
        float acc = 0.f;
        for (int f = frow_ptr[k]; f < frow_ptr[k + 1]; ++f) {
            uint32_t bb = fblk[f];
            int col = fcol[f];
            const float* B = H + (size_t)(bb & ~kTransposed) * 36;
            bool tr = (bb & kTransposed) != 0;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                float pc = it > 0 ? v.z[6 * col + c] + bf * pold[6 * col + c] : pold[6 * col + c];
                float h = tr ? B[c * 6 + a] : B[a * 6 + c];
                acc = fmaf(h, pc, acc);
            }
        }
        float pk = it > 0 ? v.z[t] + bf * pold[t] : pold[t];
        if (it > 0) pnew[t] = pk;
        v.q[t] = acc;
        pq = (double)pk * (double)acc;
    }
    pq = block_sum(pq, sh);
    if (threadIdx.x == 0) v.part_pq[blockIdx.x] = pq;
}

__global__ void __launch_bounds__(256) k_pcg_update(int nn, int it, PcgVec v) {
    __shared__ double sh[40];
    double rho = v.sc[2 * it];
    bool stop = (rho == 0.0);
    double pq = reduce_partials(v.part_pq, v.n_spmv_blocks, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) v.sc[2 * it + 1] = pq;
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    const float* p = v.p[it & 1];
    if (k < nn) {
        float r[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) r[c] = v.r[6 * k + c];
        if (!stop) {
            float alpha = (float)(rho / pq);
            double z[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                v.x[6 * k + c] = v.x[6 * k + c] + alpha * p[6 * k + c];
                r[c] = r[c] - alpha * v.q[6 * k + c];
                v.r[6 * k + c] = r[c];
            }
            apply_minv(v.Minv + (size_t)k * 36, r, z);
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                float zf = (float)z[c];
                v.z[6 * k + c] = zf;
                rz += (double)r[c] * (double)zf;
            }
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) rr += (double)r[c] * (double)r[c];
    }
    rz = block_sum(rz, sh);
    rr = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        v.part_rho[blockIdx.x] = rz;
        v.part_rr[blockIdx.x] = rr;
    }
}

// ---------------------------------------------------------------------------
// Node update T_k <- Delta_k(xi_k) o T_k and the node tables of the next step
// ---------------------------------------------------------------------------
__device__ __forceinline__ void node_tables(float4 p, Q4 r, float3 t, float4* dq, float4* cl, int k) {
    float3 u = make_float3(r.x, r.y, r.z);
    float3 c = add3(qrot(r.w, u, make_float3(p.x, p.y, p.z)), t);
    // d = 1/2 (0, t) r
    Q4 d = qmul(Q4{0.f, t.x, t.y, t.z}, r);
    dq[2 * k] = f4(r);
    dq[2 * k + 1] = make_float4(0.5f * d.w, 0.5f * d.x, 0.5f * d.y, 0.5f * d.z);
    cl[k] = make_float4(c.x, c.y, c.z, 0.f);
}

__global__ void __launch_bounds__(256) k_node_update(int nn, const float* __restrict__ x,
        const float4* __restrict__ pref, float4* __restrict__ rq, float4* __restrict__ tt,
        float4* __restrict__ dq, float4* __restrict__ cl, const double* __restrict__ part_rr, int nparts,
        IterStats* __restrict__ stats, int* __restrict__ flags) {
    __shared__ double sh[40];
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nn) {
        float3 w = make_float3(x[6 * k + 0], x[6 * k + 1], x[6 * k + 2]);
        float3 tau = make_float3(x[6 * k + 3], x[6 * k + 4], x[6 * k + 5]);
        float th = sqrtf(dot3(w, w));
        Q4 e;
        if (th < 1e-8f) {
            e = Q4{1.f, 0.5f * w.x, 0.5f * w.y, 0.5f * w.z};
        } else {
            float sn, cs;
            sincosf(0.5f * th, &sn, &cs);
            float sc = sn / th;
            e = Q4{cs, sc * w.x, sc * w.y, sc * w.z};
        }
        float en = sqrtf(((e.w * e.w + e.x * e.x) + e.y * e.y) + e.z * e.z);
        e = Q4{e.w / en, e.x / en, e.y / en, e.z / en};
        Q4 r = q4(rq[k]);
        float4 t4 = tt[k];
        float3 t = make_float3(t4.x, t4.y, t4.z);
        float4 p = pref[k];
        float3 c = add3(qrot(r.w, make_float3(r.x, r.y, r.z), make_float3(p.x, p.y, p.z)), t);
        Q4 rn = qmul(e, r);
        float nr = sqrtf(((rn.w * rn.w + rn.x * rn.x) + rn.y * rn.y) + rn.z * rn.z);
        float sgn = rn.w < 0.f ? -1.f : 1.f;
        rn = Q4{sgn * rn.w / nr, sgn * rn.x / nr, sgn * rn.y / nr, sgn * rn.z / nr};
        float3 tn = add3(add3(qrot(e.w, make_float3(e.x, e.y, e.z), sub3(t, c)), c), tau);
        bool fin = (rn.w == rn.w) && (tn.x == tn.x) && (tn.y == tn.y) && (tn.z == tn.z) && fabsf(tn.x) < INFINITY &&
                   fabsf(tn.y) < INFINITY && fabsf(tn.z) < INFINITY;
        if (!fin) atomicOr(flags, 4);
        rq[k] = f4(rn);
        tt[k] = make_float4(tn.x, tn.y, tn.z, 0.f);
        node_tables(p, rn, tn, dq, cl, k);
    }
    if (blockIdx.x == 0) {
        double rr = 0.0;
        for (int q = threadIdx.x; q < nparts; q += blockDim.x) rr += part_rr[q];
        rr = block_sum(rr, sh);
        if (threadIdx.x == 0) stats->pcg_resid = sqrt(rr);
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
void launch_depth_prep(const Cam& cam, const float* depth, float gate, float4* nmap, hipStream_t st) {
    dim3 grid((cam.W + 15) / 16, (cam.H + 15) / 16);
    hipLaunchKernelGGL(k_depth_prep, grid, dim3(256), 0, st, cam, depth, gate, nmap);
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
                     float* res, int pitch, double* part_e, int* part_n, int* corr_map, float* live_pos,
                     hipStream_t st) {
    SurfelArrays s{sv.px, sv.py, sv.pz, sv.nx, sv.ny, sv.nz, sv.idx, sv.w, sv.orig};
    CorrOut o{J, res, part_e, part_n, pitch, corr_map, live_pos};
    hipLaunchKernelGGL(k_corr_jac, dim3(corr_blocks(ns)), dim3(256), 0, st, ns, s, dq, cl, cam, z, nmap, dist2,
                       cosn, o);
}

void launch_assemble(const AssembleArgs& a, hipStream_t st) {
    AsmIn in{a.nb, a.nn, a.pitch, a.blk_row, a.col_idx, a.ent_ptr, a.ent, a.run_start, a.J, a.res, a.nbr,
             a.pref, a.rq, a.cl, a.frow_ptr, a.fcol, a.lambda, a.mu};
    AsmOut out{a.H, a.g, a.ereg};
    hipLaunchKernelGGL(k_assemble, dim3((a.nb + 3) / 4), dim3(256), 0, st, in, out);
}

void launch_jacobi(int nn, const int* row_ptr, const float* H, double* Minv, int* flags, const double* part_e,
                   const int* part_n, int nparts, const float* ereg, void* stats, hipStream_t st) {
    hipLaunchKernelGGL(k_jacobi, dim3((nn + 255) / 256), dim3(256), 0, st, nn, row_ptr, H, Minv, flags, part_e,
                       part_n, nparts, ereg, (IterStats*)stats);
}

int pcg_update_blocks(int nn) { return (nn + 255) / 256; }
int pcg_spmv_blocks(int nn) { return (6 * nn + 255) / 256; }

static PcgVec make_pcg(const PcgArgs& a) {
    PcgVec v;
    v.x = a.x; v.r = a.r; v.z = a.z; v.q = a.q; v.p[0] = a.p0; v.p[1] = a.p1;
    v.Minv = a.Minv; v.sc = a.sc; v.part_rho = a.part_rho; v.part_rr = a.part_rr; v.part_pq = a.part_pq;
    v.n_upd_blocks = pcg_update_blocks(a.nn);
    v.n_spmv_blocks = pcg_spmv_blocks(a.nn);
    return v;
}

void launch_pcg(const PcgArgs& a, int iters, hipStream_t st) {
    PcgVec v = make_pcg(a);
    int nu = pcg_update_blocks(a.nn), ns = pcg_spmv_blocks(a.nn);
    hipLaunchKernelGGL(k_pcg_init, dim3(nu), dim3(256), 0, st, a.nn, a.g, v);
    for (int it = 0; it < iters; ++it) {
        hipLaunchKernelGGL(k_pcg_spmv, dim3(ns), dim3(256), 0, st, a.nn, it, a.frow_ptr, a.fblk, a.fcol, a.H, v);
        hipLaunchKernelGGL(k_pcg_update, dim3(nu), dim3(256), 0, st, a.nn, it, v);
    }
}

void launch_node_update(int nn, const float* x, const float4* pref, float4* rq, float4* tt, float4* dq,
                        float4* cl, const double* part_rr, int nparts, void* stats, int* flags, hipStream_t st) {
    hipLaunchKernelGGL(k_node_update, dim3((nn + 255) / 256), dim3(256), 0, st, nn, x, pref, rq, tt, dq, cl,
                       part_rr, nparts, (IterStats*)stats, flags);
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

size_t iter_stats_size() { return sizeof(IterStats); }

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
