// Linear solve and node update of one Gauss-Newton iteration (Sec. 7, Sec. 8):
//
//   pcg_init     block-Jacobi preconditioner (FP64 inverses of H_kk + mu I) and
//                the start of preconditioned conjugate gradients on
//                (J^T J + mu I) delta = -g: r = -g, z = M r, p = z, x = 0
//   pcg_spmv     q = A p with p = z + beta p_old formed on the fly (one wave per
//                block row; the row's blocks, transposes written out, in ELL
//                layout)
//   pcg_update   x += alpha p, r -= alpha q, z = M r (8 lanes per node)
//   node_update  T_k <- Delta_k(xi_k) o T_k, Delta_k(x) = Exp(w)(x - c_k) + c_k + tau,
//                the reset of the index map for the next iteration and the
//                iteration's energy statistics
//
// PCG runs a fixed number of iterations and stops early only if rho = r^T z is
// exactly 0. Its scalars never leave the device: every workgroup sums the same
// per-workgroup partials (FP64) in the same order, so all workgroups take
// identical decisions and a solve is bit-reproducible.
#include <algorithm>

#include "swgn_frame.h"
#include "swgn_impl.h"
#include "swgn_launch.h"

namespace swgn {

namespace {

__device__ void update_node(const FrameDesc& a, int k) {
    const float* x = a.x + 6 * k;
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


// 8 lanes per node: lane a < 6 holds row a of [H_kk + mu I | I]; FP64
// Gauss-Jordan elimination leaves row a of the inverse. Without pivoting the
// pivots of a symmetric matrix are all positive exactly when it is positive
// definite, which is checked.
__global__ void __launch_bounds__(kSolveBlock) k_pcg_init(Batch b) {
    __shared__ double sh[40];
    const Where at = locate(b);
    const FrameDesc a = *b.d[at.s];
    const int gid = at.tile * kSolveBlock + threadIdx.x;
    const int k = gid >> 3, row = gid & 7, base = threadIdx.x & ~7;
    const bool on = (k < a.nn) && (row < 6);
    double m[12];
    const float* A = a.H + (size_t)(k < a.nn ? a.row_ptr[k] : 0) * 36;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        m[c] = on ? (double)A[row * 6 + c] : 0.0;
        m[6 + c] = (on && c == row) ? 1.0 : 0.0;
    }
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        double pr[12];
#pragma unroll
        for (int j = 0; j < 12; ++j) pr[j] = __shfl(m[j], base + c, kWave);
        const double piv = pr[c];
        ok = ok && (piv > 0.0);
        const double inv = 1.0 / (piv > 0.0 ? piv : 1.0);
        const double f = (row == c) ? 0.0 : m[c] * inv;
#pragma unroll
        for (int j = 0; j < 12; ++j) m[j] = (row == c) ? m[j] * inv : m[j] - f * pr[j];
    }
    if (k < a.nn && row == 0 && !ok) atomicOr(a.flags, 1);
    float rc = on ? -a.g[6 * k + row] : 0.f;
    double zc = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const float rj = __shfl(rc, base + j, kWave);
        const double mj = ok ? m[6 + j] : (j == row ? 1.0 : 0.0);
        zc += mj * (double)rj;
        if (on) a.Minv[(size_t)k * 36 + row * 6 + j] = mj;
    }
    double rho = 0.0, rr = 0.0;
    if (on) {
        const float zf = (float)zc;
        const int t = 6 * k + row;
        a.r[t] = rc;
        a.z[t] = zf;
        a.p0[t] = zf;
        a.x[t] = 0.f;
        rho = (double)rc * (double)zf;
        rr = (double)rc * (double)rc;
    }
    rho = block_sum(rho, sh);
    rr = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        a.part_rho[at.tile] = rho;
        a.part_rr[at.tile] = rr;
    }
}

// Products of one block row with z and with p_old: 8-lane group fl takes the
// row's slots fl, fl + 8, ...; lane sub < 6 holds row sub of the slot's block
// (one 24-byte line) and element sub of the column's z and p_old, which the
// group shares by shuffles. The row's products with z and with p_{it-1} are
// accumulated separately, so the matrix loads run before beta (a grid-wide
// sum) is known.
struct RowAcc {
    float az, ap;
};

__device__ __forceinline__ RowAcc row_products(const FrameDesc& a, const float* __restrict__ pold, int k, int lane) {
    const int sub = lane & 7, fl = lane >> 3;
    float az = 0.f, ap = 0.f;
    if (k < a.nn) {
        const uint32_t* eb = a.ell_blk + (size_t)k * a.ell_w;
        const int* ec = a.ell_col + (size_t)k * a.ell_w;
        const int base = lane & ~7;
        const int sl = sub < 6 ? sub : 0;
#pragma unroll 2
        for (int f = fl; f < a.ell_w; f += 8) {
            const uint32_t bb = eb[f];
            if (bb == 0xffffffffu) break;
            const int col = ec[f];
            const float2* B = reinterpret_cast<const float2*>(a.Hf + ((size_t)k * a.ell_w + f) * 36 + sl * 6);
            const float2 h01 = B[0], h23 = B[1], h45 = B[2];
            const float h[6] = {h01.x, h01.y, h23.x, h23.y, h45.x, h45.y};
            const float zv = a.z[6 * col + sl];
            const float pv = pold[6 * col + sl];
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const float zc = __shfl(zv, base + c, kWave);
                const float pc = __shfl(pv, base + c, kWave);
                az = fmaf(h[c], zc, az);
                ap = fmaf(h[c], pc, ap);
            }
        }
        if (sub >= 6) { az = 0.f; ap = 0.f; }
    }
    az += __shfl_xor(az, 8, kWave);
    az += __shfl_xor(az, 16, kWave);
    az += __shfl_xor(az, 32, kWave);
    ap += __shfl_xor(ap, 8, kWave);
    ap += __shfl_xor(ap, 16, kWave);
    ap += __shfl_xor(ap, 32, kWave);
    return RowAcc{az, ap};
}

// Sum of n partials in the fixed shape of a 256-thread reduction (thread t
// adds part[t], part[t + 256], ..., then the wave sums, then the 4 waves in
// order), whatever the workgroup size; result in every thread.
__device__ __forceinline__ double reduce_parts256(const double* __restrict__ part, int n, double* sh) {
    double v = 0.0;
    if (threadIdx.x < 256)
        for (int i = threadIdx.x; i < n; i += 256) v += part[i];
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x % kWave) == 0 && w < 4) sh[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < 4; ++q) t += sh[q];
        sh[32] = t;
    }
    __syncthreads();
    const double r = sh[32];
    __syncthreads();
    return r;
}

// q = A p_it with p_it = z + beta p_{it-1} (beta = 0 and p_0 = z at it = 0);
// one workgroup = 4 waves of RPW block rows each.
template <int RPW>
__global__ void __launch_bounds__(64 * kSpmvWaves) k_pcg_spmv(Batch b) {
    __shared__ double sh[40];
    __shared__ double rs[8];
    const Where at = locate(b);
    const FrameDesc a = *b.d[at.s];
    const int it = b.pcg_it;
    float* const pbuf[2] = {a.p0, a.p1};
    const float* pold = it > 0 ? pbuf[(it - 1) & 1] : pbuf[0];
    float* pcur = pbuf[it & 1];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int k0 = at.tile * kSpmvWaves * RPW + RPW * wave;
    RowAcc ra[RPW];
#pragma unroll
    for (int u = 0; u < RPW; ++u) ra[u] = row_products(a, pold, k0 + u, lane);
    const double rho = reduce_parts256(a.part_rho, solve_parts(a), sh);
    const bool stop = (rho == 0.0);
    const float beta = (it > 0 && !stop) ? (float)(rho / a.sc[(it - 1) & 1]) : 0.f;
    if (at.tile == 0 && threadIdx.x == 0) a.sc[it & 1] = rho;   // read by this iteration's update
#pragma unroll
    for (int u = 0; u < RPW; ++u) {
        const int k = k0 + u;
        double pq = 0.0;
        if (!stop && k < a.nn && lane < 6) {
            const int t = 6 * k + lane;
            const float pk = it > 0 ? a.z[t] + beta * pold[t] : pold[t];
            const float qv = ra[u].az + beta * ra[u].ap;
            if (it > 0) pcur[t] = pk;
            a.q[t] = qv;
            pq = (double)pk * (double)qv;
        }
        pq = wave_sum(pq);
        if (lane == 0) rs[RPW * wave + u] = pq;
    }
    __syncthreads();
    // partials per 4 rows, each the in-order sum of its rows' wave sums
    if (threadIdx.x < RPW) {
        const int quad = at.tile * RPW + threadIdx.x;
        if (quad < spmv_parts(a)) {
            double t = 0.0;
            for (int q = 0; q < 4; ++q) t += rs[4 * threadIdx.x + q];
            a.part_pq[quad] = t;
        }
    }
}

// x += alpha p, r -= alpha q, z = M r: 8 lanes per node, NPG nodes per lane
// group (k, k + 32, ... of the workgroup's 32 NPG).
template <int NPG>
__global__ void __launch_bounds__(kSolveBlock) k_pcg_update(Batch b) {
    __shared__ double sh[40];
    __shared__ double ws[NPG][2][4];
    const Where at = locate(b);
    const FrameDesc a = *b.d[at.s];
    const int it = b.pcg_it;
    const float* p = (it & 1) ? a.p1 : a.p0;
    const int c = threadIdx.x & 7;
    const int base = (threadIdx.x & ~7);
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    float rc[NPG], xc[NPG], pc[NPG], qc[NPG];
    double mrow[NPG][6];
#pragma unroll
    for (int u = 0; u < NPG; ++u) {
        const int k = at.tile * NPG * kSolvePart + u * kSolvePart + (threadIdx.x >> 3);
        const bool on = (k < a.nn) && (c < 6);
        const int t = 6 * k + c;
        rc[u] = xc[u] = pc[u] = qc[u] = 0.f;
        if (on) {
            rc[u] = a.r[t]; xc[u] = a.x[t]; pc[u] = p[t]; qc[u] = a.q[t];
#pragma unroll
            for (int j = 0; j < 6; ++j) mrow[u][j] = a.Minv[(size_t)k * 36 + c * 6 + j];
        } else {
#pragma unroll
            for (int j = 0; j < 6; ++j) mrow[u][j] = 0.0;
        }
    }
    const double rho = a.sc[it & 1];
    const bool stop = (rho == 0.0);
    const double pq = reduce_parts256(a.part_pq, spmv_parts(a), sh);
#pragma unroll
    for (int u = 0; u < NPG; ++u) {
        const int k = at.tile * NPG * kSolvePart + u * kSolvePart + (threadIdx.x >> 3);
        const bool on = (k < a.nn) && (c < 6);
        const int t = 6 * k + c;
        double rz = 0.0, rr = 0.0;
        float r1 = rc[u];
        if (!stop) {
            const float alpha = (float)(rho / pq);
            const float x1 = xc[u] + alpha * pc[u];
            r1 = rc[u] - alpha * qc[u];
            if (on) {
                a.x[t] = x1;
                a.r[t] = r1;
            }
            // z_c = sum_j M[c][j] r_j: the node's 6 residual entries from its lanes
            double zc = 0.0;
#pragma unroll
            for (int j = 0; j < 6; ++j) zc += mrow[u][j] * (double)__shfl(r1, base + j, kWave);
            if (on) {
                const float zf = (float)zc;
                a.z[t] = zf;
                rz = (double)r1 * (double)zf;
            }
        }
        if (on) rr = (double)r1 * (double)r1;
        rz = wave_sum(rz);
        rr = wave_sum(rr);
        if (lane == 0) {
            ws[u][0][wave] = rz;
            ws[u][1][wave] = rr;
        }
    }
    __syncthreads();
    // partials per 32 nodes, in-order sums of 4 wave sums
    if (threadIdx.x < NPG) {
        const int u = threadIdx.x;
        const int part = at.tile * NPG + u;
        if (part < solve_parts(a)) {
            double tz = 0.0, tr = 0.0;
            for (int q = 0; q < 4; ++q) { tz += ws[u][0][q]; tr += ws[u][1][q]; }
            a.part_rho[part] = tz;
            a.part_rr[part] = tr;
        }
    }
}

__global__ void __launch_bounds__(kNodeBlock) k_node_update(Batch b) {
    __shared__ double sh[40];
    const Where at = locate(b);
    const FrameDesc a = *b.d[at.s];
    const int gid = at.tile * kNodeBlock + threadIdx.x;
    if (gid < a.nn) update_node(a, gid);
    if (gid < a.npx) a.zbuf[gid] = ~0ull;     // index map of the next iteration
    if (at.tile == 0) {
        const int nparts = corr_tiles(a);
        IterStats* stats = a.stats + b.it[at.s];
        const double rr = reduce_partials(a.part_rr, solve_parts(a), sh);
        // energies at this iteration's linearisation point
        double e = 0.0, n = 0.0, er = 0.0;
        for (int t = threadIdx.x; t < nparts; t += blockDim.x) { e += a.part_e[t]; n += (double)a.part_n[t]; }
        for (int t = threadIdx.x; t < a.nn; t += blockDim.x) er += (double)a.ereg[t];
        e = block_sum(e, sh);
        n = block_sum(n, sh);
        er = block_sum(er, sh);
        if (threadIdx.x == 0) {
            stats->pcg_resid = sqrt(rr);
            stats->e_data = e;
            stats->e_reg = er;
            stats->n_corr = (int)n;
            if (!(e < INFINITY) || !(er < INFINITY)) atomicOr(a.flags, 2);
        }
    }
}

// Copies each stream's iteration statistics and failure flags to slot s of
// `out` (kStatsOutBytes per stream), so one copy brings a whole batch's back.
__global__ void __launch_bounds__(64) k_stats_out(Batch b, char* __restrict__ out) {
    const Where at = locate(b);
    const FrameDesc a = *b.d[at.s];
    int* dst = reinterpret_cast<int*>(out + (size_t)at.s * kStatsOutBytes);
    const int* src = reinterpret_cast<const int*>(a.stats);
    constexpr int nw = (int)(sizeof(IterStats) * kMaxIters / 4);
    constexpr int nr = (int)(sizeof(RigidStats) * kMaxIters / 4);
    for (int t = threadIdx.x; t < nw; t += 64) dst[t] = src[t];
    if (threadIdx.x < 4) dst[nw + threadIdx.x] = a.flags[threadIdx.x];
    const int* rsrc = reinterpret_cast<const int*>(a.rig_stats);
    for (int t = threadIdx.x; t < nr; t += 64) dst[nw + 4 + t] = rsrc[t];
}

}  // namespace

void launch_solve_stage(int stage, const Batch& b, void* stats_out, hipStream_t st) {
    const int grid = b.off[b.n];
    if (grid <= 0) return;
    switch (stage) {
        case kStPcgInit: hipLaunchKernelGGL(k_pcg_init, dim3(grid), dim3(kSolveBlock), 0, st, b); break;
        case kStSpmv:
            if (b.wide) hipLaunchKernelGGL(k_pcg_spmv<2>, dim3(grid), dim3(64 * kSpmvWaves), 0, st, b);
            else hipLaunchKernelGGL(k_pcg_spmv<1>, dim3(grid), dim3(64 * kSpmvWaves), 0, st, b);
            break;
        case kStUpdate:
            if (b.wide) hipLaunchKernelGGL(k_pcg_update<2>, dim3(grid), dim3(kSolveBlock), 0, st, b);
            else hipLaunchKernelGGL(k_pcg_update<1>, dim3(grid), dim3(kSolveBlock), 0, st, b);
            break;
        case kStNodeUpdate: hipLaunchKernelGGL(k_node_update, dim3(grid), dim3(kNodeBlock), 0, st, b); break;
        case kStStatsOut:
            hipLaunchKernelGGL(k_stats_out, dim3(grid), dim3(64), 0, st, b, static_cast<char*>(stats_out));
            break;
        default: break;
    }
}

}  // namespace swgn
