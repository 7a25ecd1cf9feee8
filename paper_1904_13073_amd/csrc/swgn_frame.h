// Per-stream frame descriptor and the batch work list of the per-frame kernels.
//
// Every per-frame kernel runs over a batch of streams in one launch: the grid
// is the concatenation of each stream's tiles, `Batch::off` is the prefix of
// tile counts, and a workgroup finds its stream by binary search over it. A
// stream's descriptor (device memory, written by the host when the stream's
// buffers change) holds its shapes, gates and every device pointer the kernels
// use. A workgroup computes from its own stream's data and its tile index in
// that stream only, so a stream's results do not depend on what else is in
// the batch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "swgn_impl.h"

namespace swgn {

constexpr int kMaxBatch = 64;
constexpr int kMaxIters = 16;
constexpr int kMaxPcg = 4096;

// Launch geometry of the per-frame kernels.
constexpr int kDepthTile = 16;        // 16 x 16 pixels per workgroup
constexpr int kWarpBlock = 256;       // surfels per workgroup
constexpr int kCorrBlock = 256;
// Surfels per correspondence pack (and at most per segment): the pack's
// Jacobian rows (28.8 KB) and the waves' output staging (10 KB) let four
// workgroups share a CU.
constexpr int kCorrPack = 232;
constexpr int kFoldGroups = 16;       // diagonal blocks per fold workgroup (16 lanes each)
constexpr int kFoldOffLanes = 4;      // lanes per off-diagonal block
constexpr int kFoldOffGroups = 256 / kFoldOffLanes;   // off-diagonal blocks per fold workgroup
constexpr int kSolveBlock = 256;      // 32 nodes x 8 lanes; the finish may take 2 nodes per lane group
constexpr int kSolveNodes = 32;       // nodes per initialisation / finishing workgroup
constexpr int kSpmvRows = 8;          // product workgroup: 8 block rows, 8 waves of 1 or 4 waves of 2
constexpr int kStepNodes = 8;         // fused PCG step: 8 nodes (one finishing wave) and their 8 rows
constexpr int kStepBlock = 64 * kStepNodes;
// Partial sums of the PCG dot products are taken per 8 nodes (r.z, r.r: one
// wave's sum) and per 8 block rows (the three products that give p.q),
// whatever the launch geometry, so every reduction has one fixed shape.
constexpr int kSolvePart = 8;
constexpr int kSpmvPart = 8;
static_assert(kSpmvRows == kSpmvPart && kStepNodes == kSpmvPart && kStepNodes == kSolvePart,
              "a product or fused-step workgroup writes exactly one partial of each kind");
constexpr int kNodeBlock = 256;
constexpr int kRigidSurfels = 1024;   // surfels per rigid-system workgroup (4 per thread)


// Per-step statistics of the rigid alignment.
struct RigidStats {
    double e;                     // sum of squared point-to-plane residuals
    int n, pad;                   // correspondences
};

// Sums per tile of the rigid alignment: 21 entries of the upper 6x6 J^T J,
// 6 of J^T r, r^T r and the correspondence count.
constexpr int kRigidSums = 29;

// Two buffers used by iteration parity. Named members rather than an array:
// a kernel's copy of the descriptor then stays in scalar registers when the
// parity is a run-time value (a select, not an indexed load).
template <class T>
struct ParityPair {
    T* b0;
    T* b1;
};

template <class T>
__host__ __device__ __forceinline__ T* by_parity(const ParityPair<T>& pp, int q) {
    // both pointers are read, then one is chosen by a mask (no address select
    // into the descriptor)
    const uintptr_t x0 = reinterpret_cast<uintptr_t>(pp.b0), x1 = reinterpret_cast<uintptr_t>(pp.b1);
    const uintptr_t m = uintptr_t(0) - uintptr_t(q & 1);
    return reinterpret_cast<T*>((x0 & ~m) | (x1 & m));
}

struct FrameDesc {
    // shapes
    int ns, nn, nb, noff, nseg, pitch, npx, ell_w;
    int npack;                    // packs: consecutive whole segments, at most kCorrPack surfels
    int64_t part_floats;          // floats of all segments' Gram sub-blocks
    int pcg_iters, debug_iter;
    int gn_iters;                 // Gauss-Newton iterations of a frame
    int jac_dtype;                // Jacobian entries kept as 0 fp32, 1 bf16, 2 fp16
    int rigid_iters;              // rigid alignment steps before the non-rigid ones
    int vis_mode;                 // 1: only stable or recently observed surfels are rendered
    int splat;                    // 1: surfels rendered as opaque discs of their radius, pairs per pixel
    float stable_conf;            // delta_stable
    int recent, t_now;            // delta_recent, current frame time
    Cam cam;
    float edge_gate, dist2, cosn, lambda, mu, pad2;
    // resident: surfels sorted by node set; orig = caller's index
    const float *px, *py, *pz, *nx, *ny, *nz;
    const int4* idx;
    const float4* w;
    const int* orig;
    float *radius, *conf;         // surfel attributes (radius, confidence, last observed frame)
    int* t_obs;
    const int* inv;               // caller index -> sorted position
    // resident: nodes
    const float4* pref;
    float4 *rq, *tt, *dq, *cl;
    const int* nbr;
    // resident: upper block pattern and the assembly / product work lists
    const int *row_ptr, *col_idx, *blk_row, *offlist, *seg_start, *ent_ptr;
    const int *pack_start, *pack_seg;   // [npack + 1] first surfel / first segment of each pack
    const uint16_t* pos4;         // [ns] positions (3 bits each) of a surfel's 4 nodes in its segment
    const uint16_t* seg_mask;     // [nseg] node pairs of the segment that share a surfel
    const uint32_t* seg_off;      // [nseg + 1] float offset of each segment's Gram sub-blocks
    const uint32_t *ent_sub, *ent_grad;   // per entry: float offset of the sub-block / J^T r piece
    const int *in_ptr, *in_list;
    const uint32_t* ell_blk;      // [nn][ell_w] upper block id (bit 31: used transposed), ~0 = padding
    const int* ell_col;           // [nn][ell_w] column node
    const int *slot_u, *slot_t;   // [nb] ELL slot of each upper block and of its transpose (-1: diagonal)
    // resident: capture of one iteration (null unless requested)
    int* dbg_corr;
    float* dbg_live;              // [6 ns]: live positions, then live normals (caller order)
    float* J;                     // [pitch][32]: 30 Jacobian entries (5 node positions), r, zero
    // workspace of a frame in flight
    float* depth;                 // copy of a host depth image
    float4* nmap;                 // (normal, depth) per pixel
    unsigned long long* zbuf;     // index map: (z bits << 32 | surfel) per pixel
    int* flags;                   // [4] failure bits of the frame
    IterStats* stats;             // [kMaxIters]
    float4 *rq_bak, *tt_bak;      // node state at the start of the frame
    float* part;                  // [part_floats] segment Gram sub-blocks, J^T r, r^T r
    float *H, *g, *ereg;          // H: upper blocks (the diagonal always, all when captured)
    float* Hf;                    // [nn][ell_w][36] full rows of J^T J + mu I, transposes written out
    double* Minv;                 // [nn][36] block-Jacobi inverses
    double* part_e;               // correspondence pass partials
    int* part_n;
    // PCG: the step x; residual r, preconditioned residual z, direction p and
    // the products u = A z, v = A p_prev, each in two buffers by iteration
    // parity (a fused step reads one while it writes the other); FP64 partial
    // sums, also by parity: r.z and r.r per 8 nodes, z.u, z.v + p.u and p.v
    // per 4 rows; sc = rho of the last two iterations
    float* x;
    ParityPair<float> r, z, p, u, v;
    double* sc;
    ParityPair<double> part_rho, part_rr, part_c;
    // rigid alignment: the transform (R row-major, t) as used by the warp
    // kernels and in FP64 for the updates, per-tile partials of the 6x6
    // system, per-step statistics
    float* rig;                   // [12]
    double* rig64;                // [12]
    double* rig_part;             // [tiles][kRigidSums]
    RigidStats* rig_stats;        // [kMaxIters]
};

// Whether sorted surfel i is rendered into the solver's index map (Sec. 7:
// stable surfels, or recently observed ones, when the stream asks for it).
__device__ __forceinline__ bool visible(const FrameDesc& d, int i) {
    // recent < 0: the recent clause is off (only stable surfels render)
    return d.vis_mode == 0 || d.conf[i] > d.stable_conf || (d.recent >= 0 && d.t_now - d.t_obs[i] <= d.recent);
}

// Tiles (workgroups) of each per-frame stage for one stream.
// kStSpmv forms the products of a PCG iteration, kStUpdate finishes one,
// kStPcgStep does both in one launch (finish of iteration i - 1, products of i).
enum Stage {
    kStDepth = 0, kStWarp, kStCorr, kStAsmSeg, kStPcgInit, kStSpmv, kStUpdate, kStNodeUpdate, kStAsmFold,
    kStRigidWarp, kStRigidSys, kStRigidSolve, kStRigidCompose, kStPcgStep, kStStatsOut, kNumStages
};
// timing slot (sw_frame_stats.stage_us) of each stage; fused PCG steps take
// slot 3 (the segment stage has no launch of its own)
inline int stage_slot(int stage) { return stage == kStPcgStep ? kStAsmSeg : stage < kStRigidCompose ? stage : 11; }

__host__ __device__ inline int cdiv(int a, int b) { return (a + b - 1) / b; }
__host__ __device__ inline int corr_tiles(const FrameDesc& d) { return d.npack; }
__host__ __device__ inline int solve_parts(const FrameDesc& d) { return cdiv(d.nn, kSolvePart); }
__host__ __device__ inline int solve_tiles(const FrameDesc& d) { return cdiv(d.nn, kSolveNodes); }
__host__ __device__ inline int spmv_parts(const FrameDesc& d) { return cdiv(d.nn, kSpmvPart); }

// Launch variant of a stage: bit 0 = tile order (kOrderXcd), bit 1 = the
// wider geometry of the stage where it has one (2 block rows per product
// wave, 2 nodes per finishing lane group), bit 2 (on kStSpmv) = PCG iterations
// as fused steps instead of product + finish launches. No variant changes any
// arithmetic.
constexpr int kVarXcd = 1;
constexpr int kVarWide = 2;
constexpr int kVarFused = 4;

inline int stage_tiles(int stage, const FrameDesc& d, int variant = 0) {
    switch (stage) {
        case kStDepth: {
            const int px = cdiv(d.cam.W, kDepthTile) * cdiv(d.cam.H, kDepthTile);
            const int nt = cdiv(d.nn, kDepthTile * kDepthTile);
            return px > nt ? px : nt;
        }
        case kStWarp: return cdiv(d.ns, kWarpBlock);
        case kStCorr: return corr_tiles(d);
        case kStAsmSeg: return 0;     // the segment Gram matrices are formed by the correspondence kernel
        case kStAsmFold: return cdiv(d.nn, kFoldGroups) + cdiv(d.noff, kFoldOffGroups);
        case kStPcgInit: return solve_tiles(d);
        case kStSpmv: return cdiv(d.nn, kSpmvRows);
        case kStUpdate: return cdiv(d.nn, (variant & kVarWide) ? 2 * kSolveNodes : kSolveNodes);
        case kStPcgStep: return cdiv(d.nn, kStepNodes);
        case kStNodeUpdate: return cdiv(d.nn > d.npx ? d.nn : d.npx, kNodeBlock);
        case kStRigidWarp: return cdiv(d.ns, kWarpBlock);
        case kStRigidSys: return cdiv(d.ns, kRigidSurfels);
        case kStRigidSolve: return cdiv(d.npx, kNodeBlock);
        case kStRigidCompose: return cdiv(d.nn, kNodeBlock);
        case kStStatsOut: return 1;
        default: return 0;
    }
}

// Work list of one launch, passed by value as a kernel argument.
struct Batch {
    int n;                        // streams
    int pcg_it;                   // PCG iteration of this launch (products of it; finish of it, or of
                                  // it - 1 in a fused step)
    int order;                    // kOrderXcd: tiles in XCD-contiguous order
    int wide;                     // the stage's wider geometry (kVarWide)
    int splat;                    // some stream renders splats (the kernels with splat code run)
    int update;                   // a stream's last PCG finish in this launch also moves its nodes
    int off[kMaxBatch + 1];       // stream s owns tiles [off[s], off[s+1])
    const FrameDesc* d[kMaxBatch];
    int8_t it[kMaxBatch];         // Gauss-Newton iteration of each stream
};

struct DepthIn {
    const float* p[kMaxBatch];    // depth image of each stream (device)
};

// Tile order of a launch. Workgroups are dealt to the 8 XCDs round-robin
// (workgroup i runs on XCD i mod 8). With kOrderXcd, XCD x takes one
// contiguous range of tiles instead of every 8th tile, so a stream's tiles
// (and the node tables, maps and blocks they touch) stay in few L2s. The
// mapping is a bijection on [0, tiles) and changes no arithmetic.
constexpr int kOrderLinear = 0;
constexpr int kOrderXcd = 1;
constexpr int kXcds = 8;

__device__ __forceinline__ int tile_of_block(int i, int tiles, int order) {
    if (order != kOrderXcd) return i;
    const int x = i % kXcds, k = i / kXcds;
    const int q = tiles / kXcds, r = tiles % kXcds;
    return x * q + (x < r ? x : r) + k;
}

struct Where {
    int s;       // stream index in the batch
    int tile;    // tile index within the stream
};

// Largest s with off[s] <= tile (streams with no tiles are skipped).
__device__ __forceinline__ Where locate(const Batch& b) {
    const int t = tile_of_block(blockIdx.x, b.off[b.n], b.order);
    int lo = 0, hi = b.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.off[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return Where{lo, t - b.off[lo]};
}

// Statistics of Gauss-Newton iteration `it` of a stream, by one workgroup of
// 256 threads: the data energy and correspondence count of its linearisation
// point (the correspondence tiles' partials), the regulariser energy (per
// node) and |r| of its last PCG residual, each a strided per-thread sum, then
// the wave sums, then the 4 waves in order; a non-finite energy sets failure
// bit 2. Runs after the iteration's node update and before the next
// iteration's correspondence kernel overwrites the partials.
__device__ __forceinline__ void iteration_stats(const FrameDesc& a, int it) {
    __shared__ double sh[16];
    const int nparts = corr_tiles(a);
    const double* prr = by_parity(a.part_rr, a.pcg_iters & 1);
    double v[4] = {0.0, 0.0, 0.0, 0.0};     // e, n, e_reg, r.r
#pragma unroll 4
    for (int t = threadIdx.x; t < nparts; t += 256) { v[0] += a.part_e[t]; v[1] += (double)a.part_n[t]; }
#pragma unroll 4
    for (int t = threadIdx.x; t < a.nn; t += 256) v[2] += (double)a.ereg[t];
#pragma unroll 4
    for (int t = threadIdx.x; t < solve_parts(a); t += 256) v[3] += prr[t];
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] = wave_sum(v[m]);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x % kWave) == 0) {
#pragma unroll
        for (int m = 0; m < 4; ++m) sh[4 * w + m] = v[m];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[4] = {0.0, 0.0, 0.0, 0.0};
        for (int q = 0; q < 4; ++q)
            for (int m = 0; m < 4; ++m) tot[m] += sh[4 * q + m];
        const double e = tot[0], n = tot[1], er = tot[2], rr = tot[3];
        IterStats* stats = a.stats + it;
        stats->pcg_resid = sqrt(rr);
        stats->e_data = e;
        stats->e_reg = er;
        stats->n_corr = (int)n;
        if (!(e < INFINITY) || !(er < INFINITY)) atomicOr(a.flags, 2);
    }
    __syncthreads();
}

// Start of PCG for one node k by a group of 8 lanes (lane `row` < 6 holds row
// `row` of H_kk + mu I in hrow and g_k[row] in gk; on = the lane carries a row
// of a node that exists): the block-Jacobi inverse by FP64 Gauss-Jordan
// elimination (no pivoting: the pivots of a symmetric matrix are all positive
// exactly when it is positive definite, which is checked; failure bit 1),
// then r_0 = -g, z_0 = M r_0, x = 0 and the direction before the first,
// p_{-1} = 0. Returns the lane's terms of r_0.z_0 and r_0.r_0.
__device__ __forceinline__ void pcg_start_lane(const FrameDesc& a, int k, int row, bool on, const float (&hrow)[6],
                                               float gk, double& rho, double& rr) {
    double m[12];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        m[c] = on ? (double)hrow[c] : 0.0;
        m[6 + c] = (on && c == row) ? 1.0 : 0.0;
    }
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        double pr[12];
#pragma unroll
        for (int j = 0; j < 12; ++j) pr[j] = bcast8(m[j], c);
        const double piv = pr[c];
        ok = ok && (piv > 0.0);
        const double inv = 1.0 / (piv > 0.0 ? piv : 1.0);
        const double f = (row == c) ? 0.0 : m[c] * inv;
#pragma unroll
        for (int j = 0; j < 12; ++j) m[j] = (row == c) ? m[j] * inv : m[j] - f * pr[j];
    }
    if (k < a.nn && row == 0 && !ok) atomicOr(a.flags, 1);
    const float rc = on ? -gk : 0.f;
    double zc = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const float rj = bcast8(rc, j);
        const double mj = ok ? m[6 + j] : (j == row ? 1.0 : 0.0);
        zc += mj * (double)rj;
        if (on) a.Minv[(size_t)k * 36 + row * 6 + j] = mj;
    }
    rho = 0.0;
    rr = 0.0;
    if (on) {
        const float zf = (float)zc;
        const int t = 6 * k + row;
        a.r.b0[t] = rc;
        a.z.b0[t] = zf;
        a.p.b1[t] = 0.f;
        a.x[t] = 0.f;
        rho = (double)rc * (double)zf;
        rr = (double)rc * (double)rc;
    }
}

// Launchers (one per kernel file); grid = b.off[b.n] workgroups.
void launch_frame_stage(int stage, const Batch& b, const DepthIn* depth, hipStream_t st);
void launch_asm_stage(int stage, const Batch& b, hipStream_t st);
void launch_solve_stage(int stage, const Batch& b, void* stats_out, hipStream_t st);

// Bytes per stream written by the statistics copy: kMaxIters IterStats, the
// failure flags, kMaxIters RigidStats.
constexpr int kStatsOutBytes = (int)(sizeof(IterStats) * kMaxIters) + 16 + (int)(sizeof(RigidStats) * kMaxIters);

}  // namespace swgn
