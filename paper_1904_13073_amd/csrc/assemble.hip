// Assembly of the Gauss-Newton system (Sec. 8: build J^T J, then solve):
//   H = sum_i J_i^T J_i + lambda sum_edges J_e^T J_e + mu I   (6x6 node-pair blocks)
//   g = sum_i J_i^T r_i + lambda sum_edges J_e^T r_e
// over the upper block pattern. Data rows come from the per-surfel Jacobians
// written by the correspondence kernel; regulariser rows (Sec. 7,
// E_regulation = sum_j sum_{m in N_j} |T_j p_j - T_m p_j|^2) are formed here
// from the node state.
//
// Work decomposition: a diagonal block (every surfel touching the node, a few
// hundred) gets a whole wave; an off-diagonal block (the surfels shared by two
// nodes, tens) gets a 16-lane row of a wave. Lanes walk the block's runs of
// surfels (surfels sharing one node set are contiguous), accumulate in
// registers with FMA, and finish with a DPP row reduction: no atomics, a fixed
// summation order, one write per block.
#include "swgn_impl.h"
#include "swgn_launch.h"

namespace swgn {

namespace {

struct AsmIn {
    int nb, nn, noff, pitch;
    const int* blk_row;
    const int* col_idx;
    const int* row_ptr;
    const int* offlist;
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
    float* H;
    float* g;
    float* ereg;
};

__device__ __forceinline__ float3 ld3(float4 a) { return make_float3(a.x, a.y, a.z); }

// y = R_m (p_j - p_m), r_jm = c_j - c_m - y
__device__ __forceinline__ void arap_edge(const AsmIn& in, int j, int m, float3& y, float3& r) {
    float3 pj = ld3(in.pref[j]), pm = ld3(in.pref[m]);
    float4 q = in.rq[m];
    y = qrot(q.x, make_float3(q.y, q.z, q.w), sub3(pj, pm));
    r = sub3(sub3(ld3(in.cl[j]), ld3(in.cl[m])), y);
}

__device__ __forceinline__ bool has_edge(const int* __restrict__ nbr, int j, int m) {
    bool e = false;
#pragma unroll
    for (int q = 0; q < 8; ++q) e |= (nbr[8 * j + q] == m);
    return e;
}

// Walk the surfels of block b's runs with `width` lanes (lane index g within
// the group) and call f(surfel, pos_a, pos_b) for each.
template <int WIDTH, class F>
__device__ __forceinline__ void for_block_surfels(const AsmIn& in, int e0, int e1, int g, F&& f) {
    for (int eb = e0; eb < e1; eb += WIDTH) {
        int j = eb + g;
        bool have = j < e1;
        uint32_t e = have ? in.ent[j] : 0u;
        int run = (int)(e >> 4);
        int st = have ? in.run_start[run] : 0;
        int len = have ? in.run_start[run + 1] - st : 0;
        int pp = (int)(e & 15u);
        int incl = len;
#pragma unroll
        for (int o = 1; o < WIDTH; o <<= 1) {
            int t = __shfl_up(incl, o, WIDTH);
            if (g >= o) incl += t;
        }
        int total = __shfl(incl, WIDTH - 1, WIDTH);
        for (int f0 = 0; f0 < total; f0 += WIDTH) {
            int fl = f0 + g;
            int lo = 0, hi = WIDTH - 1;
#pragma unroll
            for (int s = 1; s < WIDTH; s <<= 1) {
                int mid = (lo + hi) >> 1;
                int v = __shfl(incl, mid, WIDTH);
                if (v > fl) hi = mid; else lo = mid + 1;
            }
            int inc_j = __shfl(incl, lo, WIDTH);
            int len_j = __shfl(len, lo, WIDTH);
            int st_j = __shfl(st, lo, WIDTH);
            int pp_j = __shfl(pp, lo, WIDTH);
            if (fl < total) f(st_j + (fl - (inc_j - len_j)), pp_j >> 2, pp_j & 3);
        }
    }
}

__global__ void __launch_bounds__(256) k_assemble(AsmIn in, int n_diag_wg) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const size_t P = (size_t)in.pitch;
    const float lam = in.lambda;
    if ((int)blockIdx.x < n_diag_wg) {
        // ---------------- diagonal block of node k: one wave ----------------
        const int k = blockIdx.x * 4 + wave;
        if (k >= in.nn) return;
        const int b = in.row_ptr[k];
        float acc[21];   // upper triangle, row-major (a <= c)
        float gacc[6];
        float er = 0.f;
#pragma unroll
        for (int t = 0; t < 21; ++t) acc[t] = 0.f;
#pragma unroll
        for (int t = 0; t < 6; ++t) gacc[t] = 0.f;
        for_block_surfels<kWave>(in, in.ent_ptr[b], in.ent_ptr[b + 1], lane, [&](int s, int pa, int) {
            const float* Ja = in.J + (size_t)(pa * 6) * P + s;
            float x[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) x[c] = Ja[c * P];
            float rr = in.res[s];
            int t = 0;
#pragma unroll
            for (int a = 0; a < 6; ++a) {
#pragma unroll
                for (int c = a; c < 6; ++c, ++t) acc[t] = fmaf(x[a], x[c], acc[t]);
                gacc[a] = fmaf(x[a], rr, gacc[a]);
            }
        });
        // regulariser: out-edges k -> m (J_k = [0 | I]) on lanes 0..7
        if (lane < 8) {
            float3 y, r;
            arap_edge(in, k, in.nbr[8 * k + lane], y, r);
            acc[15] += lam; acc[18] += lam; acc[20] += lam;      // (3,3) (4,4) (5,5)
            gacc[3] += lam * r.x; gacc[4] += lam * r.y; gacc[5] += lam * r.z;
            er += dot3(r, r);
        }
        // in-edges j -> k (J_k = [[y]x | -I]) over the node's neighbours
        for (int f = in.frow_ptr[k] + lane; f < in.frow_ptr[k + 1]; f += kWave) {
            int j = in.fcol[f];
            if (j == k || !has_edge(in.nbr, j, k)) continue;
            float3 y, r;
            arap_edge(in, j, k, y, r);
            float yy = dot3(y, y);
            // [[|y|^2 I - y y^T, [y]x], [-[y]x, I]], upper triangle
            acc[0] += lam * (yy - y.x * y.x); acc[1] += lam * (-y.x * y.y); acc[2] += lam * (-y.x * y.z);
            acc[4] += lam * (-y.z); acc[5] += lam * (y.y);                          // (0,4) (0,5)
            acc[6] += lam * (yy - y.y * y.y); acc[7] += lam * (-y.y * y.z);
            acc[8] += lam * (y.z); acc[10] += lam * (-y.x);                         // (1,3) (1,5)
            acc[11] += lam * (yy - y.z * y.z);
            acc[12] += lam * (-y.y); acc[13] += lam * (y.x);                        // (2,3) (2,4)
            acc[15] += lam; acc[18] += lam; acc[20] += lam;
            float3 rxy = cross3(r, y);                                              // g += lambda [r x y; -r]
            gacc[0] += lam * rxy.x; gacc[1] += lam * rxy.y; gacc[2] += lam * rxy.z;
            gacc[3] -= lam * r.x; gacc[4] -= lam * r.y; gacc[5] -= lam * r.z;
        }
#pragma unroll
        for (int t = 0; t < 21; ++t) acc[t] = wave64_sum(acc[t]);
#pragma unroll
        for (int t = 0; t < 6; ++t) gacc[t] = wave64_sum(gacc[t]);
        er = wave64_sum(er);
        if (lane == 0) {
            float Hb[36];
            int t = 0;
#pragma unroll
            for (int a = 0; a < 6; ++a)
#pragma unroll
                for (int c = a; c < 6; ++c, ++t) {
                    Hb[a * 6 + c] = acc[t] + (a == c ? in.mu : 0.f);
                    Hb[c * 6 + a] = Hb[a * 6 + c];
                }
            float4* out = reinterpret_cast<float4*>(in.H + (size_t)b * 36);
#pragma unroll
            for (int v = 0; v < 9; ++v) out[v] = make_float4(Hb[4 * v], Hb[4 * v + 1], Hb[4 * v + 2], Hb[4 * v + 3]);
#pragma unroll
            for (int c = 0; c < 6; ++c) in.g[6 * k + c] = gacc[c];
            in.ereg[k] = er;
        }
        return;
    }
    // ---------------- off-diagonal blocks: 16 lanes each ----------------
    const int g = lane & 15;
    const int oi = ((int)blockIdx.x - n_diag_wg) * 16 + wave * 4 + (lane >> 4);
    const bool active = oi < in.noff;
    const int b = active ? in.offlist[oi] : 0;
    const int k = in.blk_row[b], l = in.col_idx[b];
    float acc[36];
#pragma unroll
    for (int t = 0; t < 36; ++t) acc[t] = 0.f;
    const int e0 = active ? in.ent_ptr[b] : 0, e1 = active ? in.ent_ptr[b + 1] : 0;
    for_block_surfels<16>(in, e0, e1, g, [&](int s, int pa, int pb) {
        const float* Ja = in.J + (size_t)(pa * 6) * P + s;
        const float* Jb = in.J + (size_t)(pb * 6) * P + s;
        float xa[6], xb[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) { xa[c] = Ja[c * P]; xb[c] = Jb[c * P]; }
#pragma unroll
        for (int a = 0; a < 6; ++a)
#pragma unroll
            for (int c = 0; c < 6; ++c) acc[a * 6 + c] = fmaf(xa[a], xb[c], acc[a * 6 + c]);
    });
    if (active && g == 0 && has_edge(in.nbr, k, l)) {
        // edge k -> l: J_k^T J_l = [0 0; [y]x -I]
        float3 y, r;
        arap_edge(in, k, l, y, r);
        acc[19] += lam * (-y.z); acc[20] += lam * (y.y);
        acc[24] += lam * (y.z);  acc[26] += lam * (-y.x);
        acc[30] += lam * (-y.y); acc[31] += lam * (y.x);
        acc[21] -= lam; acc[28] -= lam; acc[35] -= lam;
    }
    if (active && g == 1 && has_edge(in.nbr, l, k)) {
        // edge l -> k: J_k^T J_l = [0 -[y]x; 0 -I]
        float3 y, r;
        arap_edge(in, l, k, y, r);
        acc[4] += lam * (y.z);  acc[5] += lam * (-y.y);
        acc[9] += lam * (-y.z); acc[11] += lam * (y.x);
        acc[15] += lam * (y.y); acc[16] += lam * (-y.x);
        acc[21] -= lam; acc[28] -= lam; acc[35] -= lam;
    }
#pragma unroll
    for (int t = 0; t < 36; ++t) acc[t] = row16_sum(acc[t]);
    if (active && g == 0) {
        float4* out = reinterpret_cast<float4*>(in.H + (size_t)b * 36);
#pragma unroll
        for (int v = 0; v < 9; ++v) out[v] = make_float4(acc[4 * v], acc[4 * v + 1], acc[4 * v + 2], acc[4 * v + 3]);
    }
}

__global__ void k_offlist(int nb, const int* __restrict__ blk_row, const int* __restrict__ col_idx,
                          int* __restrict__ offlist) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    int k = blk_row[b];
    if (col_idx[b] != k) offlist[b - k - 1] = b;   // the diagonal is first in each row
}

}  // namespace

void launch_offlist(int nb, const int* blk_row, const int* col_idx, int* offlist, hipStream_t st) {
    hipLaunchKernelGGL(k_offlist, dim3((nb + 255) / 256), dim3(256), 0, st, nb, blk_row, col_idx, offlist);
}

void launch_assemble(const AssembleArgs& a, hipStream_t st) {
    AsmIn in{a.nb, a.nn, a.nb - a.nn, a.pitch, a.blk_row, a.col_idx, a.row_ptr, a.offlist, a.ent_ptr, a.ent,
             a.run_start, a.J, a.res, a.nbr, a.pref, a.rq, a.cl, a.frow_ptr, a.fcol, a.lambda, a.mu, a.H, a.g,
             a.ereg};
    int n_diag_wg = (a.nn + 3) / 4;
    int n_off_wg = (a.nb - a.nn + 15) / 16;
    hipLaunchKernelGGL(k_assemble, dim3(n_diag_wg + n_off_wg), dim3(256), 0, st, in, n_diag_wg);
}

}  // namespace swgn
