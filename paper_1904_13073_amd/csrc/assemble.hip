// Assembly of the Gauss-Newton system (Sec. 8: build J^T J, then solve):
//   H = sum_i J_i^T J_i + lambda sum_edges J_e^T J_e + mu I   (6x6 node-pair blocks)
//   g = sum_i J_i^T r_i + lambda sum_edges J_e^T r_e
// over the upper block pattern. The data term arrives as per-segment Gram
// matrices (a segment = a run of surfels with at most 5 nodes in all; the
// 6x6 sub-blocks of its node pairs and J^T r, written by the correspondence
// kernel, found through the block's entries); regulariser
// rows (Sec. 7, E_regulation = sum_j sum_{m in N_j} |T_j p_j - T_m p_j|^2) are
// formed here from the node state.
//
// A group of lanes per block (16 for a diagonal block, 4 for an off-diagonal
// one, which has few segments) sums its segments' sub-blocks in a fixed
// order, adds the regulariser terms (edges spread over the lanes) and the
// damping, and finishes with a DPP reduction over the group. No atomics;
// results are reproducible.
#include "swgn_frame.h"
#include "swgn_impl.h"
#include "swgn_launch.h"

namespace swgn {

namespace {

__device__ __forceinline__ float3 ld3(float4 a) { return make_float3(a.x, a.y, a.z); }

// y = R_m (p_j - p_m), r_jm = c_j - c_m - y
__device__ __forceinline__ void arap_edge(const FrameDesc& in, int j, int m, float3& y, float3& r) {
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


// Sum over the L lanes of a block's group (every lane ends with it): a
// 16-lane row with DPP mirror, half-mirror and two quad permutations, a quad
// with the two quad permutations.
template <int L>
__device__ __forceinline__ float group_sum(float v) {
    if constexpr (L == 16) {
        return row16_sum(v);
    } else {
        static_assert(L == 4, "groups of 16 or 4 lanes");
        v += dpp<0xB1>(v);    // quad_perm [1,0,3,2]
        v += dpp<0x4E>(v);    // quad_perm [2,3,0,1]
        return v;
    }
}

// float4 number v (a lane-dependent value in [s L, min(9, s L + L))) of the
// block (T: of its transpose), row-major; the selects keep every register
// index a compile-time constant.
template <int L, bool T>
__device__ __forceinline__ float4 pick4(const float (&acc)[36], int v, int s) {
    float r[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int v0 = s * L;
        float x = 0.f;
#pragma unroll
        for (int w = v0; w < (v0 + L < 9 ? v0 + L : 9); ++w) {
            const int q = 4 * w + e;                       // element q of the (transposed) block
            const float y = T ? acc[6 * (q % 6) + q / 6] : acc[q];
            x = (w == v0 || v == w) ? y : x;
        }
        r[e] = x;
    }
    return make_float4(r[0], r[1], r[2], r[3]);
}

// One block by a group of L lanes (lane g of the group): its segments'
// sub-blocks summed by the lanes in a fixed order, the regulariser terms
// spread over the lanes, the group sums, the damping; then the block into
// its row of the explicit rows (and its transpose into the column's row), the
// upper copy H for the diagonal (all blocks when captured), g and the
// regulariser energy for the diagonal.
template <int L>
__device__ __forceinline__ void fold_block(const FrameDesc& in, bool capture, bool active, bool diag, int b, int g,
                                           double& rho, double& rr) {
    const int k = in.blk_row[b], l = in.col_idx[b];
    const float lam = in.lambda;
    float acc[36];
    float gacc[6];
    float er = 0.f;
#pragma unroll
    for (int t = 0; t < 36; ++t) acc[t] = 0.f;
#pragma unroll
    for (int t = 0; t < 6; ++t) gacc[t] = 0.f;
    const int e0 = active ? in.ent_ptr[b] : 0, e1 = active ? in.ent_ptr[b + 1] : 0;
    for (int e = e0 + g; e < e1; e += L) {
        const float4* blk = reinterpret_cast<const float4*>(in.part + in.ent_sub[e]);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const float4 t4 = blk[q];
            acc[4 * q] += t4.x; acc[4 * q + 1] += t4.y; acc[4 * q + 2] += t4.z; acc[4 * q + 3] += t4.w;
        }
        if (diag) {
            const float* gp = in.part + in.ent_grad[e];
#pragma unroll
            for (int c = 0; c < 6; ++c) gacc[c] += gp[c];
        }
    }
    if (active && diag) {
        for (int q = g; q < 8; q += L) {      // out-edge k -> m: J_k = [0 | I]
            float3 y, r;
            arap_edge(in, k, in.nbr[8 * k + q], y, r);
            acc[21] += lam; acc[28] += lam; acc[35] += lam;
            gacc[3] += lam * r.x; gacc[4] += lam * r.y; gacc[5] += lam * r.z;
            er += dot3(r, r);
        }
        for (int f = in.in_ptr[k] + g; f < in.in_ptr[k + 1]; f += L) {   // in-edge j -> k: J_k = [[y]x | -I]
            float3 y, r;
            arap_edge(in, in.in_list[f], k, y, r);
            const float yy = dot3(y, y);
            // [[|y|^2 I - y y^T, [y]x], [-[y]x, I]]
            const float a00 = lam * (yy - y.x * y.x), a01 = lam * (-y.x * y.y), a02 = lam * (-y.x * y.z);
            const float a11 = lam * (yy - y.y * y.y), a12 = lam * (-y.y * y.z), a22 = lam * (yy - y.z * y.z);
            acc[0] += a00; acc[1] += a01; acc[2] += a02;
            acc[6] += a01; acc[7] += a11; acc[8] += a12;
            acc[12] += a02; acc[13] += a12; acc[14] += a22;
            const float sx = lam * y.x, sy = lam * y.y, sz = lam * y.z;
            // top-right [y]x = [[0,-yz,yy],[yz,0,-yx],[-yy,yx,0]], bottom-left its transpose
            acc[4] -= sz; acc[5] += sy; acc[9] += sz; acc[11] -= sx; acc[15] -= sy; acc[16] += sx;
            acc[19] += sz; acc[20] -= sy; acc[24] -= sz; acc[26] += sx; acc[30] += sy; acc[31] -= sx;
            acc[21] += lam; acc[28] += lam; acc[35] += lam;
            const float3 rxy = cross3(r, y);  // g += lambda [r x y; -r]
            gacc[0] += lam * rxy.x; gacc[1] += lam * rxy.y; gacc[2] += lam * rxy.z;
            gacc[3] -= lam * r.x; gacc[4] -= lam * r.y; gacc[5] -= lam * r.z;
        }
    } else if (active) {
        if (g == 0 && has_edge(in.nbr, k, l)) {   // edge k -> l: J_k^T J_l = [0 0; [y]x -I]
            float3 y, r;
            arap_edge(in, k, l, y, r);
            acc[19] += lam * (-y.z); acc[20] += lam * (y.y);
            acc[24] += lam * (y.z);  acc[26] += lam * (-y.x);
            acc[30] += lam * (-y.y); acc[31] += lam * (y.x);
            acc[21] -= lam; acc[28] -= lam; acc[35] -= lam;
        }
        if (g == 1 && has_edge(in.nbr, l, k)) {   // edge l -> k: J_k^T J_l = [0 -[y]x; 0 -I]
            float3 y, r;
            arap_edge(in, l, k, y, r);
            acc[4] += lam * (y.z);  acc[5] += lam * (-y.y);
            acc[9] += lam * (-y.z); acc[11] += lam * (y.x);
            acc[15] += lam * (y.y); acc[16] += lam * (-y.x);
            acc[21] -= lam; acc[28] -= lam; acc[35] -= lam;
        }
    }
#pragma unroll
    for (int t = 0; t < 36; ++t) acc[t] = group_sum<L>(acc[t]);
    if (diag) {
#pragma unroll
        for (int t = 0; t < 6; ++t) gacc[t] = group_sum<L>(gacc[t]);
        er = group_sum<L>(er);
    }
    if (active && diag) {
#pragma unroll
        for (int a = 0; a < 6; ++a) acc[7 * a] += in.mu;
        if (g == 0) {
#pragma unroll
            for (int c = 0; c < 6; ++c) in.g[6 * k + c] = gacc[c];
            in.ereg[k] = er;
        }
    }
    if (active) {
        // every lane of the group holds the block: lane g stores float4s g,
        // g + L, ... of the block into its row of the product and (off the
        // diagonal) those of the transpose into the column's row
        float* Hf = in.Hf;
#pragma unroll
        for (int s = 0; s * L < 9; ++s) {
            const int v = g + s * L;
            if (v < 9) {
                const float4 fu4 = pick4<L, false>(acc, v, s);
                reinterpret_cast<float4*>(Hf + (size_t)in.slot_u[b] * 36)[v] = fu4;
                if (diag || capture) reinterpret_cast<float4*>(in.H + (size_t)b * 36)[v] = fu4;
                if (!diag) reinterpret_cast<float4*>(Hf + (size_t)in.slot_t[b] * 36)[v] = pick4<L, true>(acc, v, s);
            }
        }
    }
    rho = 0.0;
    rr = 0.0;
    if (diag) {
        // the start of PCG for node k: lanes 0-5 of the group take the rows
        // of the block (lanes 8-15 form an 8-lane group of their own with no
        // rows); every lane holds the whole block, so a lane's row is picked
        // by selects
        const bool on = active && g < 6;
        float hrow[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            float v = acc[c];
#pragma unroll
            for (int q = 1; q < 6; ++q) v = (g == q) ? acc[6 * q + c] : v;
            hrow[c] = on ? v : 0.f;
        }
        float gk = gacc[0];
#pragma unroll
        for (int q = 1; q < 6; ++q) gk = (g == q) ? gacc[q] : gk;
        pcg_start_lane(in, active ? k : in.nn, g, on, hrow, on ? gk : 0.f, rho, rr);
    }
}

// Diagonal blocks first, one per 16-lane group (node order, kFoldGroups per
// workgroup); then the off-diagonal ones, which have few segments each, one
// per 4-lane group (kFoldOffGroups per workgroup).
__global__ void __launch_bounds__(256) k_asm_fold(Batch wl) {
    const Where at = locate(wl);
    const FrameDesc in = *wl.d[at.s];
    const bool capture = wl.it[at.s] == in.debug_iter;
    const int dtiles = cdiv(in.nn, kFoldGroups);
    double rho, rr;
    if (at.tile < dtiles) {
        __shared__ double stg[2][kFoldGroups][8];
        const int grp = threadIdx.x >> 4, g = threadIdx.x & 15;
        const int gi = at.tile * kFoldGroups + grp;
        const bool active = gi < in.nn;
        fold_block<16>(in, capture, active, true, active ? in.row_ptr[gi] : 0, g, rho, rr);
        // partials of r_0.z_0 and r_0.r_0 per 8 nodes, summed in the layout of
        // a wave of 8 nodes x 8 lanes (the start kernel's)
        if (g < 8) {
            stg[0][grp][g] = rho;
            stg[1][grp][g] = rr;
        }
        __syncthreads();
        const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
        if (wave < kFoldGroups / 8) {
            double s0 = stg[0][8 * wave + (lane >> 3)][lane & 7];
            double s1 = stg[1][8 * wave + (lane >> 3)][lane & 7];
            s0 = wave_sum(s0);
            s1 = wave_sum(s1);
            const int part = at.tile * (kFoldGroups / 8) + wave;
            if (lane == 0 && part < solve_parts(in)) {
                in.part_rho.b0[part] = s0;
                in.part_rr.b0[part] = s1;
            }
        }
    } else {
        const int gi = (at.tile - dtiles) * kFoldOffGroups + (threadIdx.x >> 2);
        const bool active = gi < in.noff;
        fold_block<kFoldOffLanes>(in, capture, active, false, active ? in.offlist[gi] : 0, threadIdx.x & 3, rho, rr);
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

void launch_asm_stage(int stage, const Batch& b, hipStream_t st) {
    const int grid = b.off[b.n];
    if (grid <= 0) return;
    if (stage == kStAsmFold) hipLaunchKernelGGL(k_asm_fold, dim3(grid), dim3(256), 0, st, b);
}

}  // namespace swgn
