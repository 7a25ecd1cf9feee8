// Linear solve and node update of one Gauss-Newton iteration (Sec. 7, Sec. 8):
//
//   PCG start    block-Jacobi preconditioner (FP64 inverses of H_kk + mu I) and
//                the start of preconditioned conjugate gradients on
//                (J^T J + mu I) delta = -g: r_0 = -g, z_0 = M r_0, x = 0
//                (pcg_start_lane: in a solve, run by the assembly fold's
//                diagonal groups; k_pcg_init runs it as a launch of its own)
//   pcg_spmv     products of iteration i: u_i = A z_i and v_i = A p_{i-1} (one
//                wave per block row; the row's blocks, transposes written out,
//                in ELL layout) and the partial sums that give p_i.q_i once
//                beta_i is known
//   pcg_finish   finish of iteration i: beta_i, alpha_i, p_i = z_i + beta_i p_{i-1},
//                x += alpha p_i, r -= alpha (u_i + beta_i v_i), z = M r
//                (8 lanes per node)
//   pcg_step     finish of iteration i - 1 and products of iteration i in one
//                launch: the products re-form their columns' z_i and p_{i-1}
//   node update  T_k <- Delta_k(xi_k) o T_k, Delta_k(x) = Exp(w)(x - c_k) + c_k + tau,
//                and the reset of the index map for the next iteration: done
//                by a stream's last PCG finish (fused step or finish launch),
//                by k_node_update only for streams without PCG iterations;
//                the iteration's energy statistics are summed by the next
//                iteration's warp launch or, for the last, the statistics copy
//
// This is standard preconditioned CG (the same iterates in exact arithmetic)
// with the application of beta deferred: the product kernel needs only
// vectors of the previous finish, so a finish and the next products can share
// a launch. PCG runs a fixed number of iterations and stops early only if
// rho = r^T z is exactly 0. Its scalars never leave the device: every
// workgroup sums the same partials (FP64) in the same order, so all workgroups
// take identical decisions and a solve is bit-reproducible, with fused steps
// or without.
#include <algorithm>

#include "swgn_frame.h"
#include "swgn_impl.h"
#include "swgn_launch.h"

namespace swgn {

namespace {


__device__ void update_node_x(const FrameDesc& a, int k, const float (&x)[6]) {
    float3 w = make_float3(x[0], x[1], x[2]);
    float3 tau = make_float3(x[3], x[4], x[5]);
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
    Q4 r = q4(a.rq[k]);
    float4 t4 = a.tt[k];
    float3 t = make_float3(t4.x, t4.y, t4.z);
    float4 p = a.pref[k];
    float3 c = add3(qrot(r.w, make_float3(r.x, r.y, r.z), make_float3(p.x, p.y, p.z)), t);
    Q4 rn = qmul(e, r);
    float nr = sqrtf(((rn.w * rn.w + rn.x * rn.x) + rn.y * rn.y) + rn.z * rn.z);
    float sg = rn.w < 0.f ? -1.f : 1.f;
    rn = Q4{sg * rn.w / nr, sg * rn.x / nr, sg * rn.y / nr, sg * rn.z / nr};
    float3 tn = add3(add3(qrot(e.w, make_float3(e.x, e.y, e.z), sub3(t, c)), c), tau);
    bool fin = fabsf(rn.w) <= 1.f && fabsf(tn.x) < INFINITY && fabsf(tn.y) < INFINITY && fabsf(tn.z) < INFINITY;
    if (!fin) atomicOr(a.flags, 4);
    a.rq[k] = f4(rn);
    a.tt[k] = make_float4(tn.x, tn.y, tn.z, 0.f);
    node_tables(p, rn, tn, a.dq, a.cl, k);
}

__device__ void update_node(const FrameDesc& a, int k) {
    float x[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) x[j] = a.x[6 * k + j];
    update_node_x(a, k, x);
}

// Index map of the next iteration: tile `tile` of a launch with `ntiles`
// tiles for the stream clears its share of the pixels.
__device__ __forceinline__ void reset_index_map(const FrameDesc& a, int tile, int ntiles) {
    const int chunk = cdiv(a.npx, ntiles);
    const int p0 = tile * chunk, p1 = min(a.npx, p0 + chunk);
    for (int p = p0 + (int)threadIdx.x; p < p1; p += (int)blockDim.x) a.zbuf[p] = ~0ull;
}

// The node update of a stream's last PCG finish, inside the finishing lane
// group (lane c holds component c of x_k): the group's 6 entries of x to
// every lane, lane 0 moves node k.
__device__ __forceinline__ void update_from_lanes(const FrameDesc& a, int k, int c, float xc) {
    float x[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) x[j] = bcast8(xc, j);
    if (c == 0 && k < a.nn) update_node_x(a, k, x);
}


// The start of PCG (pcg_start_lane), 8 lanes per node, 32 nodes per
// workgroup, as a launch of its own: the solve forms it inside the assembly
// fold; this launch serves stage replays.
__global__ void __launch_bounds__(kSolveBlock) k_pcg_init(Batch b) {
    const Where at = locate(b);
    const FrameDesc a = *b.d[at.s];
    const int gid = at.tile * kSolveBlock + threadIdx.x;
    const int k = gid >> 3, row = gid & 7;
    const int lane = threadIdx.x % kWave;
    const bool on = (k < a.nn) && (row < 6);
    float hrow[6];
    const float* A = a.H + (size_t)(k < a.nn ? a.row_ptr[k] : 0) * 36;
#pragma unroll
    for (int c = 0; c < 6; ++c) hrow[c] = on ? A[row * 6 + c] : 0.f;
    const float gk = on ? a.g[6 * k + row] : 0.f;
    double rho, rr;
    pcg_start_lane(a, k, row, on, hrow, gk, rho, rr);
    // partials per 8 nodes: one wave's sums
    rho = wave_sum(rho);
    rr = wave_sum(rr);
    const int part = gid / kWave;
    if (lane == 0 && part < solve_parts(a)) {
        a.part_rho.b0[part] = rho;
        a.part_rr.b0[part] = rr;
    }
}

// Scalars that finish PCG iteration k (rho_k = r_k.z_k from the node partials,
// p_k.q_k from the three row products, rho_{k-1} from the ring):
//   beta_k = rho_k / rho_{k-1} (0 at k = 0), p_k = z_k + beta_k p_{k-1},
//   q_k = A p_k = u_k + beta_k v_k,
//   p_k.q_k = z.u + beta (z.v + p.u) + beta^2 p.v,   alpha_k = rho_k / p_k.q_k.
// rho_k = 0 stops the iteration: alpha = beta = 0 leave x, r and z as they are.
// Every workgroup sums the same partials in the same order, so all take the
// same scalars; workgroup 0 of the stream keeps rho_k for the next finish.
struct PcgScalars {
    float alpha, beta;
};

// Four sums of partials at once, each in the fixed shape of a 256-thread
// reduction whatever the workgroup size (thread t < 256 adds part[t],
// part[t + 256], ..., then the wave sums, then the 4 waves in order): one
// pass of loads and one exchange instead of four.
struct Sum4 {
    double s[4];
};

__device__ __forceinline__ Sum4 reduce4_parts256(const double* __restrict__ p0, int n0,
                                                 const double* __restrict__ p123, int n123, double* sh) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (threadIdx.x < 256) {
        for (int i = threadIdx.x; i < n0; i += 256) v[0] += p0[i];
        for (int i = threadIdx.x; i < n123; i += 256) {
            v[1] += p123[i];
            v[2] += p123[n123 + i];
            v[3] += p123[2 * n123 + i];
        }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] = wave_sum(v[m]);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x % kWave) == 0 && w < 4) {
#pragma unroll
        for (int m = 0; m < 4; ++m) sh[4 * w + m] = v[m];
    }
    __syncthreads();
    Sum4 r;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        double t = 0.0;
        for (int q = 0; q < 4; ++q) t += sh[4 * q + m];
        r.s[m] = t;
    }
    __syncthreads();
    return r;
}

__device__ __forceinline__ PcgScalars pcg_scalars(const FrameDesc& a, int k, bool keep, double* sh) {
    const int par = k & 1, nsp = spmv_parts(a);
    const Sum4 t = reduce4_parts256(by_parity(a.part_rho, par), solve_parts(a), by_parity(a.part_c, par), nsp, sh);
    const double rho = t.s[0], c1 = t.s[1], c2 = t.s[2], c3 = t.s[3];
    const bool stop = (rho == 0.0);
    const float beta = (k > 0 && !stop) ? (float)(rho / a.sc[(k - 1) & 1]) : 0.f;
    const double bd = (double)beta;
    const double pq = (c1 + bd * c2) + (bd * bd) * c3;
    const float alpha = stop ? 0.f : (float)(rho / pq);
    if (keep && threadIdx.x == 0) a.sc[par] = rho;
    return PcgScalars{alpha, beta};
}

// The finish of iteration k for one component of one node (8 lanes per node,
// component c = lane & 7 < 6, lanes 6 and 7 carry zeros): p_k, r_{k+1},
// z_{k+1} = M r_{k+1} (FP64 sum of the node's 6 entries, read by shuffles
// within the lane group) and x_{k+1}. A fused step repeats the same
// operations for the nodes of its rows' columns, so both agree bit for bit.
struct Finished {
    float p, r, z, x;
};

__device__ __forceinline__ Finished finish_lane(float zk, float pprev, float uk, float vk, float rk, float xk,
                                                const double (&mrow)[6], PcgScalars s, int base) {
    Finished f;
    f.p = zk + s.beta * pprev;
    const float q = uk + s.beta * vk;
    f.x = xk + s.alpha * f.p;
    f.r = rk - s.alpha * q;
    double zc = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) zc += mrow[j] * (double)bcast8(f.r, j);
    f.z = (float)zc;
    return f;
}

// Finish of iteration k = b.pcg_it: x_{k+1}, r_{k+1}, z_{k+1}, p_k; partials
// of rho_{k+1} and r_{k+1}.r_{k+1}. NPG nodes per lane group (k, k + 32, ...
// of the workgroup's 32 NPG); each wave's 8 nodes give one partial. A
// stream's last finish (b.update) also moves its nodes by x and clears its
// share of the index map.
template <int NPG>
__global__ void __launch_bounds__(kSolveBlock) k_pcg_finish(Batch b) {
    __shared__ double sh[40];
    const Where at = locate(b);
    const FrameDesc a = *b.d[at.s];
    const int k = b.pcg_it, cur = k & 1, nxt = cur ^ 1;
    const int c = threadIdx.x & 7, base = threadIdx.x & ~7;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    float zc[NPG], pc[NPG], uc[NPG], vc[NPG], rc[NPG], xc[NPG];
    double mrow[NPG][6];
#pragma unroll
    for (int g = 0; g < NPG; ++g) {
        const int n = at.tile * NPG * kSolveNodes + g * kSolveNodes + (threadIdx.x >> 3);
        const bool on = (n < a.nn) && (c < 6);
        const int t = 6 * n + c;
        zc[g] = pc[g] = uc[g] = vc[g] = rc[g] = xc[g] = 0.f;
#pragma unroll
        for (int j = 0; j < 6; ++j) mrow[g][j] = 0.0;
        if (on) {
            zc[g] = by_parity(a.z, cur)[t]; pc[g] = by_parity(a.p, nxt)[t]; uc[g] = by_parity(a.u, cur)[t]; vc[g] = by_parity(a.v, cur)[t];
            rc[g] = by_parity(a.r, cur)[t]; xc[g] = a.x[t];
#pragma unroll
            for (int j = 0; j < 6; ++j) mrow[g][j] = a.Minv[(size_t)n * 36 + c * 6 + j];
        }
    }
    const PcgScalars s = pcg_scalars(a, k, at.tile == 0, sh);
#pragma unroll
    for (int g = 0; g < NPG; ++g) {
        const int n = at.tile * NPG * kSolveNodes + g * kSolveNodes + (threadIdx.x >> 3);
        const bool on = (n < a.nn) && (c < 6);
        const int t = 6 * n + c;
        const Finished f = finish_lane(zc[g], pc[g], uc[g], vc[g], rc[g], xc[g], mrow[g], s, base);
        double rz = 0.0, rr = 0.0;
        if (on) {
            a.x[t] = f.x;
            by_parity(a.r, nxt)[t] = f.r;
            by_parity(a.z, nxt)[t] = f.z;
            by_parity(a.p, cur)[t] = f.p;
            rz = (double)f.r * (double)f.z;
            rr = (double)f.r * (double)f.r;
        }
        rz = wave_sum(rz);
        rr = wave_sum(rr);
        const int part = (at.tile * NPG * kSolveNodes + g * kSolveNodes) / kSolvePart + wave;
        if (lane == 0 && part < solve_parts(a)) {
            by_parity(a.part_rho, nxt)[part] = rz;
            by_parity(a.part_rr, nxt)[part] = rr;
        }
        if (b.update && k == a.pcg_iters - 1) update_from_lanes(a, n, c, f.x);
    }
    if (b.update && k == a.pcg_iters - 1) reset_index_map(a, at.tile, cdiv(a.nn, NPG * kSolveNodes));
}

// Products of one block row with z_i and with p_{i-1} (u_i and v_i of the
// row): 8-lane group fl takes the row's slots fl, fl + 8, ...; lane sub < 6
// holds row sub of the slot's block (one 24-byte line) and element sub of the
// column's vectors, which the group shares by shuffles. With FUSED, the
// column's z_i and p_{i-1} are formed here from its iteration-(i-1) state by
// the finish operations (same order, same rounding) instead of being read.
// The first two slots of each group are loaded by row_prefetch (which a fused
// step issues before its scalars are known); row_products goes on from there.
struct RowAcc {
    float u, v;
};

struct SlotData {
    int n;                        // slots in use: 0, 1 or 2 (slots fl and fl + 8)
    float h[2][6];                // the block's row sub (zero for an unused slot)
    float c[2][5];                // column: z_{i-1}, p_{i-2}, u_{i-1}, v_{i-1}, r_{i-1} (FUSED), else z_i, p_{i-1}
    double m[2][6];               // FUSED: row sub of the column's inverse
};

template <bool FUSED>
__device__ __forceinline__ void load_slot(const FrameDesc& a, int i, int row, int f, int col, int sub, float (&h)[6],
                                          float (&cv)[5], double (&m)[6]) {
    const int cur = i & 1, prv = cur ^ 1;
    const int sl = sub < 6 ? sub : 0;
    const float2* B = reinterpret_cast<const float2*>(a.Hf + ((size_t)row * a.ell_w + f) * 36 + sl * 6);
    const float2 h01 = gld2(B), h23 = gld2(B + 1), h45 = gld2(B + 2);
    h[0] = h01.x; h[1] = h01.y; h[2] = h23.x; h[3] = h23.y; h[4] = h45.x; h[5] = h45.y;
    const int t = 6 * col + sl;
    if (FUSED) {
        cv[0] = gld(by_parity(a.z, prv) + t);
        cv[1] = gld(by_parity(a.p, cur) + t);
        cv[2] = gld(by_parity(a.u, prv) + t);
        cv[3] = gld(by_parity(a.v, prv) + t);
        cv[4] = gld(by_parity(a.r, prv) + t);
#pragma unroll
        for (int j = 0; j < 6; ++j) m[j] = gld(a.Minv + (size_t)col * 36 + sl * 6 + j);
    } else {
        cv[0] = gld(by_parity(a.z, cur) + t);
        cv[1] = gld(by_parity(a.p, prv) + t);
    }
}

// The first two slots of each lane group are loaded without a branch (a
// padding slot reads slot 0's column and an in-bounds block, and its block
// is zeroed), so that no load waits for the padding test: the block loads
// go out at once, the column loads after the column index.
template <bool FUSED>
__device__ __forceinline__ void row_prefetch(const FrameDesc& a, int i, int row, int lane, SlotData& sd) {
    const int sub = lane & 7, fl = lane >> 3;
    sd.n = 0;
    if (row >= a.nn) return;
    const uint32_t* eb = a.ell_blk + (size_t)row * a.ell_w;
    const int* ec = a.ell_col + (size_t)row * a.ell_w;
    bool use[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int f = fl + 8 * q;
        const int fc = f < a.ell_w ? f : 0;
        use[q] = f < a.ell_w && gld(eb + fc) != 0xffffffffu;
        load_slot<FUSED>(a, i, row, fc, gld(ec + fc), sub, sd.h[q], sd.c[q], sd.m[q]);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int c = 0; c < 6; ++c) sd.h[q][c] = use[q] ? sd.h[q][c] : 0.f;
    // slots are used from the front (padding only at a row's end)
    sd.n = use[1] ? 2 : (use[0] ? 1 : 0);
}

// the column's z and p of one slot (FUSED: its finish of iteration i - 1)
template <bool FUSED>
__device__ __forceinline__ void slot_vectors(const float (&cv)[5], const double (&m)[6], int sub, int base,
                                             PcgScalars s, float& zv, float& pv) {
    if (FUSED) {
        double mr[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) mr[j] = sub < 6 ? m[j] : 0.0;
        const bool on = sub < 6;
        const Finished fin = finish_lane(on ? cv[0] : 0.f, on ? cv[1] : 0.f, on ? cv[2] : 0.f, on ? cv[3] : 0.f,
                                         on ? cv[4] : 0.f, 0.f, mr, s, base);
        zv = fin.z;
        pv = fin.p;
    } else {
        zv = cv[0];
        pv = cv[1];
    }
}

__device__ __forceinline__ void slot_products(const float (&h)[6], float zv, float pv, int base, float& au,
                                              float& av) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const float zc = bcast8(zv, c);
        const float pc = bcast8(pv, c);
        au = fmaf(h[c], zc, au);
        av = fmaf(h[c], pc, av);
    }
}

template <bool FUSED>
__device__ __forceinline__ RowAcc row_products(const FrameDesc& a, int i, int row, int lane, PcgScalars s,
                                               const SlotData& sd) {
    const int sub = lane & 7, fl = lane >> 3;
    const int base = lane & ~7;
    float au = 0.f, av = 0.f;
    if (row < a.nn) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (q >= sd.n) break;
            float zv, pv;
            slot_vectors<FUSED>(sd.c[q], sd.m[q], sub, base, s, zv, pv);
            slot_products(sd.h[q], zv, pv, base, au, av);
        }
        if (sd.n == 2) {
            const uint32_t* eb = a.ell_blk + (size_t)row * a.ell_w;
            const int* ec = a.ell_col + (size_t)row * a.ell_w;
            for (int f = fl + 16; f < a.ell_w; f += 8) {
                if (eb[f] == 0xffffffffu) break;
                float h[6], cv[5];
                double m[6];
                load_slot<FUSED>(a, i, row, f, ec[f], sub, h, cv, m);
                float zv, pv;
                slot_vectors<FUSED>(cv, m, sub, base, s, zv, pv);
                slot_products(h, zv, pv, base, au, av);
            }
        }
        if (sub >= 6) { au = 0.f; av = 0.f; }
    }
    au += xchg<8>(au);
    au += xchg<16>(au);
    au += xchg<32>(au);
    av += xchg<8>(av);
    av += xchg<16>(av);
    av += xchg<32>(av);
    return RowAcc{au, av};
}

// Sum of a value that only lanes 0-5 hold (every other lane holds +0): the
// value the wave butterfly 32, 16, ..., 1 gives, valid in lanes 0-7. Its
// first three steps only add +0, which turns -0 into +0, as one addition of
// +0 does.
__device__ __forceinline__ double low6_sum(double v) {
    v += 0.0;
    v += xchg<4>(v);
    v += xchg<2>(v);
    v += xchg<1>(v);
    return v;
}

// Stores u_i, v_i of a row and returns the row's three products
// (z.u, z.v + p.u, p.v over its 6 entries, summed over lanes 0-5; valid in
// lane 0).
struct RowProducts {
    double c1, c2, c3;
};

__device__ __forceinline__ RowProducts store_row(const FrameDesc& a, int i, int row, int lane, RowAcc ra,
                                                 float zo, float po) {
    double c1 = 0.0, c2 = 0.0, c3 = 0.0;
    if (row < a.nn && lane < 6) {
        const int t = 6 * row + lane;
        by_parity(a.u, i & 1)[t] = ra.u;
        by_parity(a.v, i & 1)[t] = ra.v;
        c1 = (double)zo * (double)ra.u;
        c2 = (double)zo * (double)ra.v + (double)po * (double)ra.u;
        c3 = (double)po * (double)ra.v;
    }
    return RowProducts{low6_sum(c1), low6_sum(c2), low6_sum(c3)};
}

// Partial of a workgroup's 8 rows (kSpmvPart): the in-order sum of its rows'
// products, one value for each of the three.
__device__ __forceinline__ void store_row_parts(const FrameDesc& a, int i, int part, const double (*rs)[3]) {
    if (threadIdx.x < 3 && part < spmv_parts(a)) {
        const int m = threadIdx.x;
        double t = 0.0;
        for (int w = 0; w < kSpmvPart; ++w) t += rs[w][m];
        by_parity(a.part_c, i & 1)[m * spmv_parts(a) + part] = t;
    }
}

// Products of iteration i = b.pcg_it from z_i and p_{i-1} as stored; one
// workgroup = 8 block rows, 8 / RPW waves of RPW rows each.
template <int RPW>
__global__ void __launch_bounds__(64 * kSpmvRows / RPW) k_pcg_spmv(Batch b) {
    __shared__ double rs[kSpmvRows][3];
    const Where at = locate(b);
    const FrameDesc a = *b.d[at.s];
    const int i = b.pcg_it;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int k0 = at.tile * kSpmvRows + RPW * wave;
    RowAcc ra[RPW];
#pragma unroll
    for (int g = 0; g < RPW; ++g) {
        SlotData sd;
        row_prefetch<false>(a, i, k0 + g, lane, sd);
        ra[g] = row_products<false>(a, i, k0 + g, lane, PcgScalars{0.f, 0.f}, sd);
    }
#pragma unroll
    for (int g = 0; g < RPW; ++g) {
        const int row = k0 + g;
        float zo = 0.f, po = 0.f;
        if (row < a.nn && lane < 6) {
            zo = by_parity(a.z, i & 1)[6 * row + lane];
            po = by_parity(a.p, (i & 1) ^ 1)[6 * row + lane];
        }
        const RowProducts rp = store_row(a, i, row, lane, ra[g], zo, po);
        if (lane == 0) {
            rs[RPW * wave + g][0] = rp.c1;
            rs[RPW * wave + g][1] = rp.c2;
            rs[RPW * wave + g][2] = rp.c3;
        }
    }
    __syncthreads();
    store_row_parts(a, i, at.tile, rs);
}

// One fused PCG step i = b.pcg_it >= 1 over 8 nodes: wave 0 finishes iteration
// i - 1 for them (as k_pcg_finish), then, if i < pcg_iters, wave w forms the
// products of iteration i for row 8 tile + w, computing the columns' z_i and
// p_{i-1} itself (row_products<true>). One launch per PCG iteration instead of
// two, at the cost of re-reading each column's state and inverse. The
// stream's last step (i = pcg_iters, with b.update) moves its nodes and
// clears its share of the index map instead of forming products.
__global__ void __launch_bounds__(kStepBlock) k_pcg_step(Batch b) {
    __shared__ double sh[40];
    __shared__ double rs[kStepNodes][3];
    __shared__ float own_z[kStepNodes * 8], own_p[kStepNodes * 8];
    const Where at = locate(b);
    const FrameDesc a = *b.d[at.s];
    const int i = b.pcg_it, k = i - 1, cur = k & 1, nxt = cur ^ 1;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int n0 = at.tile * kStepNodes;
    const bool prod = i < a.pcg_iters;     // uniform: false at this stream's last finish
    // loads first (they do not depend on the scalars): the finishing wave's
    // own nodes, every wave's first two slots of its row
    const int c = lane & 7, base = lane & ~7;
    const int n = n0 + (lane >> 3);
    const bool on = (wave == 0) && (n < a.nn) && (c < 6);
    const int t = 6 * n + c;
    float zk = 0.f, pp = 0.f, uk = 0.f, vk = 0.f, rk = 0.f, xk = 0.f;
    double mrow[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) mrow[j] = 0.0;
    if (on) {
        zk = by_parity(a.z, cur)[t]; pp = by_parity(a.p, nxt)[t]; uk = by_parity(a.u, cur)[t];
        vk = by_parity(a.v, cur)[t]; rk = by_parity(a.r, cur)[t];
        xk = a.x[t];
#pragma unroll
        for (int j = 0; j < 6; ++j) mrow[j] = a.Minv[(size_t)n * 36 + c * 6 + j];
    }
    const int row = n0 + wave;
    SlotData sd;
    sd.n = 0;
    if (prod) row_prefetch<true>(a, i, row, lane, sd);
    const PcgScalars s = pcg_scalars(a, k, at.tile == 0, sh);
    if (wave == 0) {
        const Finished f = finish_lane(zk, pp, uk, vk, rk, xk, mrow, s, base);
        double rz = 0.0, rr = 0.0;
        if (on) {
            a.x[t] = f.x;
            by_parity(a.r, nxt)[t] = f.r;
            by_parity(a.z, nxt)[t] = f.z;
            by_parity(a.p, cur)[t] = f.p;
            rz = (double)f.r * (double)f.z;
            rr = (double)f.r * (double)f.r;
        }
        own_z[lane] = on ? f.z : 0.f;
        own_p[lane] = on ? f.p : 0.f;
        rz = wave_sum(rz);
        rr = wave_sum(rr);
        if (lane == 0 && n0 / kSolvePart < solve_parts(a)) {
            by_parity(a.part_rho, nxt)[n0 / kSolvePart] = rz;
            by_parity(a.part_rr, nxt)[n0 / kSolvePart] = rr;
        }
        if (!prod && b.update) update_from_lanes(a, n, c, f.x);
    }
    if (!prod) {
        if (b.update) reset_index_map(a, at.tile, cdiv(a.nn, kStepNodes));
        return;
    }
    __syncthreads();
    const RowAcc ra = row_products<true>(a, i, row, lane, s, sd);
    const float zo = lane < 6 ? own_z[wave * 8 + lane] : 0.f;
    const float po = lane < 6 ? own_p[wave * 8 + lane] : 0.f;
    const RowProducts rp = store_row(a, i, row, lane, ra, zo, po);
    if (lane == 0) {
        rs[wave][0] = rp.c1;
        rs[wave][1] = rp.c2;
        rs[wave][2] = rp.c3;
    }
    __syncthreads();
    store_row_parts(a, i, n0 / kSpmvPart, rs);
}

// The node update of streams without PCG iterations (x = 0) and the reset
// of their index map; streams with PCG iterations are updated by their last
// finish.
__global__ void __launch_bounds__(kNodeBlock) k_node_update(Batch b) {
    const Where at = locate(b);
    const FrameDesc a = *b.d[at.s];
    const int gid = at.tile * kNodeBlock + threadIdx.x;
    if (gid < a.nn) update_node(a, gid);
    if (gid < a.npx) a.zbuf[gid] = ~0ull;     // index map of the next iteration
}

// Sums the statistics of each stream's last Gauss-Newton iteration (the
// earlier ones were summed by the warp launch of the next iteration) and
// copies its iteration statistics and failure flags to slot s of `out`
// (kStatsOutBytes per stream), so one copy brings a whole batch's back.
__global__ void __launch_bounds__(256) k_stats_out(Batch b, char* __restrict__ out) {
    const Where at = locate(b);
    const FrameDesc a = *b.d[at.s];
    if (a.gn_iters > 0) iteration_stats(a, a.gn_iters - 1);
    int* dst = reinterpret_cast<int*>(out + (size_t)at.s * kStatsOutBytes);
    const int* src = reinterpret_cast<const int*>(a.stats);
    constexpr int nw = (int)(sizeof(IterStats) * kMaxIters / 4);
    constexpr int nr = (int)(sizeof(RigidStats) * kMaxIters / 4);
    for (int t = threadIdx.x; t < nw; t += blockDim.x) dst[t] = src[t];
    if (threadIdx.x < 4) dst[nw + threadIdx.x] = a.flags[threadIdx.x];
    const int* rsrc = reinterpret_cast<const int*>(a.rig_stats);
    for (int t = threadIdx.x; t < nr; t += blockDim.x) dst[nw + 4 + t] = rsrc[t];
}

}  // namespace

void launch_solve_stage(int stage, const Batch& b, void* stats_out, hipStream_t st) {
    const int grid = b.off[b.n];
    if (grid <= 0) return;
    switch (stage) {
        case kStPcgInit: hipLaunchKernelGGL(k_pcg_init, dim3(grid), dim3(kSolveBlock), 0, st, b); break;
        case kStSpmv:
            if (b.wide) hipLaunchKernelGGL(k_pcg_spmv<2>, dim3(grid), dim3(64 * kSpmvRows / 2), 0, st, b);
            else hipLaunchKernelGGL(k_pcg_spmv<1>, dim3(grid), dim3(64 * kSpmvRows), 0, st, b);
            break;
        case kStUpdate:
            if (b.wide) hipLaunchKernelGGL(k_pcg_finish<2>, dim3(grid), dim3(kSolveBlock), 0, st, b);
            else hipLaunchKernelGGL(k_pcg_finish<1>, dim3(grid), dim3(kSolveBlock), 0, st, b);
            break;
        case kStPcgStep: hipLaunchKernelGGL(k_pcg_step, dim3(grid), dim3(kStepBlock), 0, st, b); break;
        case kStNodeUpdate: hipLaunchKernelGGL(k_node_update, dim3(grid), dim3(kNodeBlock), 0, st, b); break;
        case kStStatsOut:
            hipLaunchKernelGGL(k_stats_out, dim3(grid), dim3(256), 0, st, b, static_cast<char*>(stats_out));
            break;
        default: break;
    }
}

}  // namespace swgn
