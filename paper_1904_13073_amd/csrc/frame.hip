// Per-frame kernels of the Gauss-Newton warp-field solve (Sec. 7), part 1:
//
//   depth_prep   normal map of the depth image (Sec. 5); resets the index map
//   warp_zbuf    dual-quaternion warp of every surfel (Sec. 3, Eq. 1-2) and
//                a 64-bit atomic-min z-buffer of (z bits, surfel index) (Sec. 7)
//   corr_gram    projective correspondence, point-to-plane residual, its exact
//                Jacobian with respect to the 4 node twists, and per segment
//                of surfels sharing a node set the Gram matrix of [J | r]
// plus node-state conversions and capture helpers. Assembly is in
// assemble.hip, the linear solve and node update in solve.hip. The per-frame
// kernels take a batch of streams (one work list, see swgn_frame.h).
//
// Sums are taken in a fixed order everywhere, so a frame solve is
// bit-reproducible run to run.
#include "swgn_frame.h"
#include "swgn_impl.h"
#include "swgn_launch.h"

namespace swgn {

// ---------------------------------------------------------------------------
// Depth preprocessing: normal map by central differences (Sec. 5).
// nmap = (n, d) where the normal is defined, (0, 0, 0, 0) elsewhere. Also
// resets the index map and the failure flags and keeps the node state the
// frame starts from.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_depth_prep(Batch b, DepthIn in) {
    const Where at = locate(b);
    const FrameDesc d = *b.d[at.s];
    const float* __restrict__ depth = in.p[at.s];
    const int gid = at.tile * 256 + threadIdx.x;
    if (at.tile == 0 && threadIdx.x < 4) d.flags[threadIdx.x] = 0;
    if (at.tile == 0 && threadIdx.x < 12) {
        // the frame's rigid alignment starts from the identity
        const float e = (threadIdx.x == 0 || threadIdx.x == 4 || threadIdx.x == 8) ? 1.f : 0.f;
        d.rig[threadIdx.x] = e;
        d.rig64[threadIdx.x] = (double)e;
    }
    if (gid < d.nn) {
        d.rq_bak[gid] = d.rq[gid];
        d.tt_bak[gid] = d.tt[gid];
    }
    const Cam cam = d.cam;
    const int gx = cdiv(cam.W, kDepthTile);
    if (at.tile >= gx * cdiv(cam.H, kDepthTile)) return;
    const int x = (at.tile % gx) * kDepthTile + (threadIdx.x & 15);
    const int y = (at.tile / gx) * kDepthTile + (threadIdx.x >> 4);
    if (x >= cam.W || y >= cam.H) return;
    const int W = cam.W;
    d.zbuf[y * W + x] = ~0ull;   // index map of the first iteration
    float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
    if (x > 0 && y > 0 && x < cam.W - 1 && y < cam.H - 1) {
        float dc = depth[y * W + x];
        float dU = depth[(y - 1) * W + x], dD = depth[(y + 1) * W + x];
        float dL = depth[y * W + x - 1], dR = depth[y * W + x + 1];
        const float gate = d.edge_gate;
        bool ok = depth_ok(dc) && depth_ok(dU) && depth_ok(dD) && depth_ok(dL) && depth_ok(dR);
        if (ok) {
            ok = fabsf(dU - dc) <= gate && fabsf(dD - dc) <= gate && fabsf(dL - dc) <= gate &&
                 fabsf(dR - dc) <= gate;
        }
        if (ok) {
            float3 vU = backproject(cam, x, y - 1, dU), vD = backproject(cam, x, y + 1, dD);
            float3 vL = backproject(cam, x - 1, y, dL), vR = backproject(cam, x + 1, y, dR);
            float3 a = sub3(vD, vU);   // V(x, y+1) - V(x, y-1)
            float3 bb = sub3(vR, vL);  // V(x+1, y) - V(x-1, y)
            float c0 = a.y * bb.z - a.z * bb.y;
            float c1 = a.z * bb.x - a.x * bb.z;
            float c2 = a.x * bb.y - a.y * bb.x;
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
    d.nmap[y * W + x] = out;
}

__device__ __forceinline__ unsigned long long zkey(float z, int orig) {
    return ((unsigned long long)__float_as_uint(z) << 32) | (unsigned long long)(unsigned)orig;
}

// Splats (Sec. 7: the live surfels rendered as opaque discs). A surfel whose
// centre projects to pixel (ux, uy) is tried on the box ux +- h, uy +- h,
// h = min(4, ceil(fx r / z)); the ray of pixel u is d = ((u_x - cx)/fx,
// (u_y - cy)/fy, 1) and covers it when n . d != 0, t = (n . v)/(n . d) > 0 and
// |t d - v|^2 <= r^2, at depth t. A surfel of radius 0 (or less) is an
// unsized point at its centre pixel.
constexpr int kSplatMaxPx = 4;

__device__ __forceinline__ int splat_half(const Cam& c, float r, float z) {
    return (int)fminf((float)kSplatMaxPx, ceilf((c.fx * r) / z));
}

__device__ __forceinline__ void splat_render(const FrameDesc& d, float3 v, float3 n, float r, int ux, int uy,
                                             int org) {
    if (!(r > 0.f)) {
        atomicMin(&d.zbuf[uy * d.cam.W + ux], zkey(v.z, org));
        return;
    }
    const int h = splat_half(d.cam, r, v.z);
    const float nv = (n.x * v.x + n.y * v.y) + n.z * v.z;
    const float r2 = r * r;
    for (int oy = -h; oy <= h; ++oy) {
        const int y = uy + oy;
        if (y < 0 || y >= d.cam.H) continue;
        const float dy = ((float)y - d.cam.cy) / d.cam.fy;
        for (int ox = -h; ox <= h; ++ox) {
            const int x = ux + ox;
            if (x < 0 || x >= d.cam.W) continue;
            const float dx = ((float)x - d.cam.cx) / d.cam.fx;
            const float nd = (n.x * dx + n.y * dy) + n.z;
            if (nd == 0.f) continue;
            const float t = nv / nd;
            if (!(t > 0.f)) continue;
            const float ex = t * dx - v.x, ey = t * dy - v.y, ez = t - v.z;
            const float e2 = (ex * ex + ey * ey) + ez * ez;
            if (e2 <= r2) atomicMin(&d.zbuf[y * d.cam.W + x], zkey(t, org));
        }
    }
}

// ---------------------------------------------------------------------------
// Warp + index map
// ---------------------------------------------------------------------------
// SPLAT: a launch with a splat stream (the point rule's launches carry none of
// the splat code)
template <bool SPLAT>
__global__ void __launch_bounds__(kWarpBlock) k_warp_zbuf(Batch b) {
    static_assert(kWarpBlock == 256, "the statistics sums have the shape of a 256-thread workgroup");
    const Where at = locate(b);
    const FrameDesc d = *b.d[at.s];
    // the previous iteration's statistics, before this iteration's
    // correspondence launch overwrites its partials
    if (at.tile == 0 && b.it[at.s] >= 1) iteration_stats(d, b.it[at.s] - 1);
    const int i = at.tile * kWarpBlock + threadIdx.x;
    if (i >= d.ns || !visible(d, i)) return;     // (the correspondence test needs the surfel in the map)
    float3 v = make_float3(d.px[i], d.py[i], d.pz[i]);
    if (SPLAT && d.splat) {
        const float3 n = make_float3(d.nx[i], d.ny[i], d.nz[i]);
        const Warp ws = warp_surfel(d.idx[i], d.w[i], v, n, d.dq);
        int sx, sy;
        if (!ws.ok || !project(d.cam, ws.v, sx, sy)) return;
        splat_render(d, ws.v, ws.n, d.radius[i], sx, sy, d.orig[i]);
        return;
    }
    Warp wp = warp_surfel(d.idx[i], d.w[i], v, make_float3(0.f, 0.f, 0.f), d.dq);
    if (!wp.ok) return;
    int ux, uy;
    if (!project(d.cam, wp.v, ux, uy)) return;
    atomicMin(&d.zbuf[uy * d.cam.W + ux], zkey(wp.v.z, d.orig[i]));
}

// ---------------------------------------------------------------------------
// Correspondence, residual, Jacobian and the segment Gram matrices.
//
// A tile is a pack of whole segments (consecutive surfels, at most 256; a
// segment is a run of surfels whose nodes number at most 5 in all). Each
// thread forms its surfel's row [J | r] in LDS: node block k at the position
// of its node in the segment's ascending node list (pos4), r in column 30.
// Then each wave takes segments of the pack and sums the 31 x 31 Gram matrix
// [J | r]^T [J | r] over the segment's surfels with the 32x32x2 FP32 MFMA,
// the sum over surfels being the MFMA's k dimension (two surfels per
// instruction; the A and B operands are the same register: lane = component,
// half-wave = surfel). The 6x6 sub-blocks of the node pairs that share a
// surfel (seg_mask), J^T r and r^T r are stored for the block fold. Jacobian
// rows leave the chip only when an iteration is captured.
// ---------------------------------------------------------------------------
// LDS row stride in floats: 31 entries (J at 5 node positions, r), odd so
// that a row per lane is conflict-free. The MFMA reads 32 columns per row;
// column 31 runs into the next row (or the slack after the last one) and
// only feeds Gram entries with an index of 31, which are discarded.
constexpr int kRowPad = 31;
constexpr int kStageFloats = 576;    // per wave: a segment's whole output (at most 36 x 15 + 32 floats)
constexpr int kStageSlots = kStageFloats + kWave;   // and one discard word per lane

// Code of accumulator element t of lane l in a segment's Gram tile (element
// G[i][j], j = l % 32, i = (t / 4) * 8 + (l / 32) * 4 + t % 4): for a node-pair
// block (i, j < 30, pa = i / 6 <= pb = j / 6) its pair bit
// 5 pa - pa (pa - 1) / 2 + pb - pa (bits 0-3) and its position
// (i % 6) * 6 + j % 6 in the 6x6 sub-block (bits 4-9); for J^T r and r^T r
// (j = 30, i <= 30) bit field 15 and i; 0xffff for elements not kept.
struct GramCodes {
    uint16_t c[kWave][16];
};

constexpr GramCodes make_gram_codes() {
    GramCodes g{};
    for (int l = 0; l < kWave; ++l)
        for (int t = 0; t < 16; ++t) {
            const int i = (t / 4) * 8 + (l / 32) * 4 + t % 4, j = l % 32;
            uint16_t code = 0xffff;
            if (i < 30 && j < 30) {
                const int pa = i / 6, pb = j / 6;
                if (pa <= pb) code = (uint16_t)((5 * pa - pa * (pa - 1) / 2 + pb - pa) | (((i % 6) * 6 + j % 6) << 4));
            } else if (j == 30 && i <= 30) {
                code = (uint16_t)(15 | (i << 4));
            }
            g.c[l][t] = code;
        }
    return g;
}

__constant__ GramCodes kGramCodes = make_gram_codes();

typedef float f32x16 __attribute__((ext_vector_type(16)));


// d r / d xi_k for the 4 nodes of a matched surfel: the closed form of
// N^T dF/db(b; v) w_k s_k M(q_k, c_k). With P = N c_r, Q = N c_d, PV = P (0,v)
// and a_k = w_k s_k / |b_r|:
//   d r / d tau_k   = a_k vec(P r_k*)
//   d r / d omega_k = a_k [vec(P d_k*) - vec(W r_k*) - c_k x vec(P r_k*)],
//   W = PV + Q + (N . v') c_r   (vec(x y*) is linear in x).
// No integer decision depends on these values, so multiply-adds may fuse here.
// Quaternion helpers of the Jacobian, with multiply-adds allowed to fuse.
__device__ __forceinline__ Q4 qmul_c(Q4 a, Q4 b) {
#pragma clang fp contract(fast)
    Q4 r;
    r.w = a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z;
    r.x = a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y;
    r.y = a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x;
    r.z = a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w;
    return r;
}
__device__ __forceinline__ float3 vec_mul_conj_c(Q4 x, Q4 y) {
#pragma clang fp contract(fast)
    return make_float3(y.w * x.x - x.w * y.x - (x.y * y.z - x.z * y.y),
                       y.w * x.y - x.w * y.y - (x.z * y.x - x.x * y.z),
                       y.w * x.z - x.w * y.z - (x.x * y.y - x.y * y.x));
}

__device__ __forceinline__ void jacobian_rows(const FrameDesc& d, int4 id, float4 w4, float3 v, float3 N,
                                              const Warp& wp, float (&Jw)[4][3], float (&Jt)[4][3]) {
#pragma clang fp contract(fast)
    const Q4 Nq = {0.f, N.x, N.y, N.z};
    const Q4 P = qmul_c(Nq, wp.cr);
    const Q4 Qd = qmul_c(Nq, wp.cd);
    const Q4 PV = qmul_c(P, Q4{0.f, v.x, v.y, v.z});
    const float ndv = N.x * wp.v.x + N.y * wp.v.y + N.z * wp.v.z;
    const Q4 W = {PV.w + Qd.w + ndv * wp.cr.w, PV.x + Qd.x + ndv * wp.cr.x, PV.y + Qd.y + ndv * wp.cr.y,
                  PV.z + Qd.z + ndv * wp.cr.z};
    const int ids[4] = {id.x, id.y, id.z, id.w};
    const float wk[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const Q4 rk = q4(gld4(d.dq + 2 * ids[k]));
        const Q4 dk = q4(gld4(d.dq + 2 * ids[k] + 1));
        const float4 c4 = gld4(d.cl + ids[k]);
        const float a = wk[k] * wp.sgn[k] * wp.inv_beta;
        const float3 h = vec_mul_conj_c(P, rk);
        const float3 g1 = vec_mul_conj_c(P, dk);
        const float3 gW = vec_mul_conj_c(W, rk);
        // c_k x h
        const float cx = c4.y * h.z - c4.z * h.y, cy = c4.z * h.x - c4.x * h.z, cz = c4.x * h.y - c4.y * h.x;
        Jw[k][0] = a * (g1.x - gW.x - cx);
        Jw[k][1] = a * (g1.y - gW.y - cy);
        Jw[k][2] = a * (g1.z - gW.z - cz);
        Jt[k][0] = a * h.x;
        Jt[k][1] = a * h.y;
        Jt[k][2] = a * h.z;
    }
}

// Jacobian entry as stored: fp32, or rounded to nearest-even bf16 / fp16 and
// held in an fp32 register (products and sums stay fp32).
__device__ __forceinline__ float keep_jac(float v, int dtype) {
    if (dtype == 1) {
        uint32_t u = __float_as_uint(v);
        if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
        return __uint_as_float(u & 0xffff0000u);
    }
    if (dtype == 2) return (float)(_Float16)v;
    return v;
}

// Splat pairs of one surfel: every pair row is [N_p^T D | r_p] = a_p^T E with
// a_p = (N_p, r_p) and E = diag(D, 1), D the 3 x 30 Jacobian of the warped
// position, so the pairs' Gram sum is E^T (sum_p a_p a_p^T) E = E^T R^T R E for
// the 4 x 4 triangular factor R of the stacked a_p: at most four rows
// [J(R_j) | R_j3] (J is linear in the normal) carry all of a surfel's pairs.
// R is built by inserting the a_p one at a time: the first unused row takes
// what is left of a_p as it is (so a single pair's row is its own exactly);
// a used row is rotated with a_p in the plane of their j-th entries (Givens),
// which keeps R^T R + a a^T.
__device__ __forceinline__ void factor_insert(float (&R)[4][4], int used, float w0, float w1, float w2,
                                              float w3) {
    float w[4] = {w0, w1, w2, w3};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (used <= j) {
#pragma unroll
            for (int k = j; k < 4; ++k) R[j][k] = w[k];
            return;
        }
        if (w[j] == 0.f) continue;
        const float rad = sqrtf(R[j][j] * R[j][j] + w[j] * w[j]);
        if (!(rad > 0.f)) continue;
        const float c = R[j][j] / rad, s = w[j] / rad;
#pragma unroll
        for (int k = j; k < 4; ++k) {
            const float a = R[j][k], e = w[k];
            R[j][k] = c * a + s * e;
            w[k] = c * e - s * a;
        }
        w[j] = 0.f;
    }
}

// A row in LDS (slot: the thread's own, or a compacted one): node block k at
// its node's position in the segment (threads past the pack capacity are never
// live and keep no row).
__device__ __forceinline__ void put_row(const FrameDesc& d, float* rows, int slot, bool live, int i,
                                        float (&Jw)[4][3], float (&Jt)[4][3], float r) {
    if (slot >= kCorrPack) return;
    float* row = &rows[slot * kRowPad];
    const int p4 = live ? (int)gld(d.pos4 + i) : (0 | (1 << 3) | (2 << 6) | (3 << 9));
    const int jd = d.jac_dtype;          // uniform: one branch for the whole row
    if (jd != 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Jw[k][c] = keep_jac(Jw[k][c], jd);
                Jt[k][c] = keep_jac(Jt[k][c], jd);
            }
    }
    int used = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int pos = (p4 >> (3 * k)) & 7;
        used |= 1 << pos;
        float* o = row + pos * 6;
        o[0] = Jw[k][0]; o[1] = Jw[k][1]; o[2] = Jw[k][2];
        o[3] = Jt[k][0]; o[4] = Jt[k][1]; o[5] = Jt[k][2];
    }
    // the segment's fifth node position, if the surfel does not touch it
#pragma unroll
    for (int pos = 0; pos < 5; ++pos)
        if (!(used & (1 << pos))) {
#pragma unroll
            for (int c = 0; c < 6; ++c) row[pos * 6 + c] = 0.f;
        }
    row[30] = r;
}

// The tile statistics: sum of squared residuals (FP64) and pair count. Also
// zeroes the slack after the last row, read as column 31 (whose products are
// dropped). A block-wide barrier.
__device__ __forceinline__ void tile_sums(const FrameDesc& d, float* rows, double* sh, int* shi, int tile,
                                          double e_own, int npair) {
    if (threadIdx.x == kCorrBlock - 1) {
#pragma unroll
        for (int c = 0; c < 8; ++c) rows[kCorrPack * kRowPad + c] = 0.f;
    }
    const double e = block_sum(e_own, sh);
    const int cnt = wave_sumi(npair);
    if ((threadIdx.x % kWave) == 0) shi[threadIdx.x / kWave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int c = 0;
        for (int q = 0; q < (int)(blockDim.x / kWave); ++q) c += shi[q];
        gst(d.part_e + tile, e);
        gst(d.part_n + tile, c);
    }
}

// A captured iteration's rows, as whole 128-byte lines, two rows per store.
__device__ __forceinline__ void capture_rows(const FrameDesc& d, const float* rows, int p0, int p1) {
    {
        const int lane = threadIdx.x % kWave, base = (threadIdx.x / kWave) * kWave;
        float* dst = d.J + (size_t)(p0 + base) * 32;
        const int nrow = min(kWave, p1 - p0 - base);
#pragma nounroll
        for (int q = 0; q < kWave / 2; ++q) {
            const int rr = 2 * q + (lane >> 5), c = lane & 31;
            if (rr < nrow) dst[rr * 32 + c] = c < 31 ? rows[(base + rr) * kRowPad + c] : 0.f;
        }
    }
}

// Extra splat rows before thread t of the pack: counts 0..3 per thread held as
// two ballot bit planes per wave (planes[w], planes[4 + w]).
__device__ __forceinline__ int extra_before(const unsigned long long* planes, int t) {
    const int w = t / kWave, l = t % kWave;
    int c = 0;
    for (int q = 0; q < w; ++q) c += __popcll(planes[q]) + 2 * __popcll(planes[4 + q]);
    if (w < kCorrBlock / kWave) {
        const unsigned long long lm = l ? (~0ull >> (kWave - l)) : 0ull;
        c += __popcll(planes[w] & lm) + 2 * __popcll(planes[4 + w] & lm);
    }
    return c;
}

// Segment Gram matrices of the pack's rows, one wave per segment. Accumulator
// element t of lane l is G[i][j], j = l % 32, i = (t / 4) * 8 + (l / 32) * 4 +
// t % 4. The output slot of each element: the rank of its node pair among the
// segment's pairs x 36 + position in the 6x6 sub-block; J^T r and r^T r after
// the sub-blocks. The whole output is staged in LDS and stored as whole lines;
// with `more` (later splat rounds) segments without a marked row are skipped
// and the sums are added to the stored ones (the same lanes stored those words);
// with `planes` the rows are the compacted extra rows from slot `base` on, a
// segment's being those of its surfels in order.
__device__ __forceinline__ void segment_grams(const FrameDesc& d, const float* rows, float4* stage, int tile, int p0,
                                              const unsigned long long* more,
                                              const unsigned long long* planes = nullptr, int base = 0) {
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int comp = lane & 31, half = lane >> 5;
    const int g0 = gld(d.pack_seg + tile), g1 = gld(d.pack_seg + tile + 1);
    // the descriptor's pointers read once (the stores below could alias it)
    const int* seg_start = d.seg_start;
    const uint16_t* seg_mask = d.seg_mask;
    const uint32_t* seg_off = d.seg_off;
    float* part = d.part;
    float* sg = reinterpret_cast<float*>(stage);
    // this lane's 16 accumulator elements: the pair's bit as a mask (bit 31
    // for J^T r and r^T r, which follow the sub-blocks; 0 for an element that
    // is not kept) and the offset. An element's output slot is then
    // 36 x (pairs of the segment below its pair) + offset, where the pairs
    // below bit 31 are all of them; a dropped element goes to the lane's
    // discard word, so every element is one unconditional LDS store.
    uint32_t bm[16];
    int off[16];
    {
        const uint4* codes = reinterpret_cast<const uint4*>(kGramCodes.c[lane]);
        const uint4 q0 = codes[0], q1 = codes[1];
        const uint32_t cw[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const uint32_t code = (cw[t >> 1] >> (16 * (t & 1))) & 0xffffu;
            const uint32_t bit = code & 15u;
            bm[t] = code == 0xffffu ? 0u : (bit == 15u ? 0x80000000u : (1u << bit));
            off[t] = (int)(code >> 4);
        }
    }
    for (int seg = g0 + wave; seg < g1; seg += kCorrBlock / kWave) {
        int s0 = gld(seg_start + seg) - p0, s1 = gld(seg_start + seg + 1) - p0;
        if (planes != nullptr) {
            s0 = min(max(extra_before(planes, s0) - base, 0), kCorrPack);
            s1 = min(max(extra_before(planes, s1) - base, 0), kCorrPack);
            if (s0 == s1) continue;                            // uniform over the wave
        } else if (more != nullptr) {
            bool any = false;
            for (int m = s0 + lane; m < s1; m += kWave) any |= ((more[m / kWave] >> (m % kWave)) & 1ull) != 0;
            if (__ballot(any) == 0) continue;                  // uniform over the wave
        }
        const uint32_t mask = gld(seg_mask + seg);          // (issued before the sums)
        float4* out = reinterpret_cast<float4*>(part + gld(seg_off + seg));
        f32x16 acc;
#pragma unroll
        for (int t = 0; t < 16; ++t) acc[t] = 0.f;
        for (int m0 = s0; m0 < s1; m0 += 16) {
            float v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int sr = m0 + 2 * q + half;   // surfel of this half-wave
                const float e = rows[(sr < s1 ? sr : s0) * kRowPad + comp];   // (a row of the segment)
                v[q] = sr < s1 ? e : 0.f;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(v[q], v[q], acc, 0, 0, 0);
        }
        const int npr = __builtin_popcount(mask);
        const int size = 36 * npr + 32;
        const uint32_t mk = mask | 0x80000000u;
        // the whole output staged in LDS, then stored as whole float4 lines
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int sl = 36 * __builtin_popcount(mask & (bm[t] - 1u)) + off[t];
            sg[(mk & bm[t]) != 0u ? sl : kStageFloats + lane] = acc[t];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (more != nullptr || planes != nullptr) {
            for (int q = lane; q < size / 4; q += kWave) {
                const float4 a = gld4(out + q), c4 = stage[q];
                gst4(out + q, make_float4(a.x + c4.x, a.y + c4.y, a.z + c4.z, a.w + c4.w));
            }
        } else {
            for (int q = lane; q < size / 4; q += kWave) gst4(out + q, stage[q]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// A captured iteration's live surfel (caller order): position in dbg_live[0,
// 3 ns), normal in dbg_live[3 ns, 6 ns); NaN for a surfel without a valid blend
__device__ __forceinline__ void capture_live(const FrameDesc& d, int org, const Warp& wp) {
    const float nanv = __int_as_float(0x7fc00000);
    float* lp = d.dbg_live + 3 * (size_t)org;
    float* ln = d.dbg_live + 3 * ((size_t)d.ns + org);
    lp[0] = wp.ok ? wp.v.x : nanv;
    lp[1] = wp.ok ? wp.v.y : nanv;
    lp[2] = wp.ok ? wp.v.z : nanv;
    ln[0] = wp.ok ? wp.n.x : nanv;
    ln[1] = wp.ok ? wp.n.y : nanv;
    ln[2] = wp.ok ? wp.n.z : nanv;
}

// SPLAT: a launch with a splat stream (the point rule's launches carry none of
// the splat code)
template <bool SPLAT>
__global__ void __launch_bounds__(kCorrBlock, 4) k_corr_gram(Batch b) {
    __shared__ double sh[40];
    __shared__ int shi[16];
    __shared__ unsigned long long planes[2 * (kCorrBlock / kWave)];   // splat: extra rows per surfel
    __shared__ float rows[kCorrPack * kRowPad + 8];
    __shared__ float4 stage4[kCorrBlock / kWave][kStageSlots / 4];
    const Where at = locate(b);
    const FrameDesc& d = *b.d[at.s];
    const bool capture = (b.it[at.s] == d.debug_iter) && d.dbg_corr != nullptr;
    const int p0 = gld(d.pack_start + at.tile), p1 = gld(d.pack_start + at.tile + 1);
    const int i = p0 + (int)threadIdx.x;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const bool live = i < p1;
    float r = 0.f;
    float Jw[4][3], Jt[4][3];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) { Jw[k][c] = 0.f; Jt[k][c] = 0.f; }
    // the match decisions as one predicate (no nested branches, so the zero
    // rows of unmatched lanes are formed once); lanes past the pack take its
    // last surfel and are masked, lanes that fail early read pixel 0
    const int ic = live ? i : p1 - 1;
    const int4 id = gld4(d.idx + ic);
    const int org = gld(d.orig + ic);
    const float4 w4 = gld4(d.w + ic);
    const float3 v = make_float3(gld(d.px + ic), gld(d.py + ic), gld(d.pz + ic));
    const float3 n = make_float3(gld(d.nx + ic), gld(d.ny + ic), gld(d.nz + ic));
    const Warp wp = warp_surfel(id, w4, v, n, d.dq);
    int ux, uy;
    const bool in = project(d.cam, wp.v, ux, uy);
    bool ok = live & wp.ok & in;
    if (SPLAT && d.splat) {                                    // uniform: a workgroup is one stream's
        // the pixels this surfel won (index part of the key) that have a
        // normal and pass the gates, in row-major order of its box, reduced
        // to the factor R of their rows (a_p = (N_p, r_p))
        if (live && capture) capture_live(d, org, wp);
        int npair = 0;
        double e_own = 0.0;
        float R[4][4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int k = 0; k < 4; ++k) R[j][k] = 0.f;
        if (ok) {
            const float rr = d.radius[ic];
            const int h = rr > 0.f ? splat_half(d.cam, rr, wp.v.z) : 0;
            const unsigned* zw = reinterpret_cast<const unsigned*>(d.zbuf);   // index half of a key: its low word
            for (int oy = -h; oy <= h; ++oy) {
                const int y = uy + oy;
                if (y < 0 || y >= d.cam.H) continue;
                // the row's index words loaded together, then the pixels this
                // surfel won visited left to right
                unsigned won = 0;
                unsigned wv[2 * kSplatMaxPx + 1];
#pragma unroll
                for (int c = 0; c <= 2 * kSplatMaxPx; ++c) {
                    const int x = ux - h + c;
                    const bool inb = c <= 2 * h && x >= 0 && x < d.cam.W;
                    wv[c] = inb ? zw[2 * (y * d.cam.W + x)] : 0xffffffffu;
                }
#pragma unroll
                for (int c = 0; c <= 2 * kSplatMaxPx; ++c) won |= (wv[c] == (unsigned)org) ? 1u << c : 0u;
                while (won != 0u) {
                    const int c = __builtin_ctz(won);
                    won &= won - 1u;
                    const int x = ux - h + c;
                    const int u = y * d.cam.W + x;
                    const float4 q = d.nmap[u];
                    if (!(q.w > 0.f)) continue;
                    const float3 dq3 = sub3(wp.v, backproject(d.cam, x, y, q.w));
                    const float q2 = (dq3.x * dq3.x + dq3.y * dq3.y) + dq3.z * dq3.z;
                    const float3 Nq = make_float3(q.x, q.y, q.z);
                    if (!(q2 < d.dist2) || !(dot3(wp.n, Nq) > d.cosn)) continue;
                    const float rp = dot3(Nq, dq3);
                    factor_insert(R, npair, Nq.x, Nq.y, Nq.z, rp);
                    e_own += (double)rp * (double)rp;
                    ++npair;
                    if (capture) d.dbg_corr[u] = org;
                }
            }
        }
        tile_sums(d, rows, sh, shi, at.tile, e_own, npair);
        // round 0: row 0 of the factor of every surfel with a pair
        {
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) { Jw[k][c] = 0.f; Jt[k][c] = 0.f; }
            r = 0.f;
            if (npair > 0) {
                r = R[0][3];
                int i2 = i;
                asm volatile("" : "+v"(i2));                     // (not kept from the scan)
                const int4 id2 = d.idx[i2];
                const float4 w42 = d.w[i2];
                const float3 v2 = make_float3(d.px[i2], d.py[i2], d.pz[i2]);
                const float3 n2 = make_float3(d.nx[i2], d.ny[i2], d.nz[i2]);
                const Warp w2 = warp_surfel(id2, w42, v2, n2, d.dq);
                jacobian_rows(d, id2, w42, v2, make_float3(R[0][0], R[0][1], R[0][2]), w2, Jw, Jt);
            }
            put_row(d, rows, threadIdx.x, live, i, Jw, Jt, r);
            __syncthreads();
            if (capture) capture_rows(d, rows, p0, p1);
            segment_grams(d, rows, stage4[wave], at.tile, p0, nullptr);
        }
        // the surfels' further factor rows (1 to 3 each), compacted in surfel
        // order into the rows, so that a segment's are contiguous; their Gram
        // sums are added in one more pass over the segments
        const int extra = live ? max(0, min(npair, 4) - 1) : 0;
        {
            const unsigned long long e0 = __ballot((extra & 1) != 0), e1 = __ballot((extra & 2) != 0);
            if (lane == 0) { planes[wave] = e0; planes[4 + wave] = e1; }
        }
        __syncthreads();                                       // (round 0's rows are read too)
        const int total = extra_before(planes, kCorrBlock);
        const int slot = extra_before(planes, threadIdx.x);
        // in chunks of the pack's row capacity (one chunk unless a pack has
        // more extra rows than surfels)
#pragma nounroll
        for (int base = 0; base < total; base += kCorrPack) {
            if (base > 0) __syncthreads();                     // the previous chunk's rows are read
            if (extra > 0 && slot + extra > base && slot < base + kCorrPack) {
                int i2 = i;
                asm volatile("" : "+v"(i2));                     // (not kept from the scan)
                const int4 id2 = d.idx[i2];
                const float4 w42 = d.w[i2];
                const float3 v2 = make_float3(d.px[i2], d.py[i2], d.pz[i2]);
                const float3 n2 = make_float3(d.nx[i2], d.ny[i2], d.nz[i2]);
                const Warp w2 = warp_surfel(id2, w42, v2, n2, d.dq);
#pragma nounroll
                for (int j = 1; j <= extra; ++j) {
                    const int sl = slot + j - 1 - base;
                    if (sl < 0 || sl >= kCorrPack) continue;
                    const float ny = j == 1 ? R[1][1] : 0.f;
                    const float nz = j == 1 ? R[1][2] : (j == 2 ? R[2][2] : 0.f);
                    const float rj = j == 1 ? R[1][3] : (j == 2 ? R[2][3] : R[3][3]);
                    jacobian_rows(d, id2, w42, v2, make_float3(0.f, ny, nz), w2, Jw, Jt);
                    put_row(d, rows, sl, live, i, Jw, Jt, rj);
                }
            }
            __syncthreads();
            segment_grams(d, rows, stage4[wave], at.tile, p0, nullptr, planes, base);
        }
        return;
    }
    const int pix = ok ? uy * d.cam.W + ux : 0;
    ok = ok & (gld(d.zbuf + pix) == zkey(wp.v.z, org));   // (loaded beside the normal map)
    const float4 nm = gld4(d.nmap + pix);
    ok = ok & (nm.w > 0.f);
    const float3 V = backproject(d.cam, ux, uy, nm.w);
    const float3 dv = sub3(wp.v, V);
    const float d2 = (dv.x * dv.x + dv.y * dv.y) + dv.z * dv.z;
    const float3 N = make_float3(nm.x, nm.y, nm.z);
    const bool matched = ok & (d2 < d.dist2) & (dot3(wp.n, N) > d.cosn);
    if (matched) {
        r = dot3(N, dv);
        jacobian_rows(d, id, w4, v, N, wp, Jw, Jt);
    }
    if (threadIdx.x < kCorrPack) {
        // the row: node block k at its node's position in the segment
        // (threads past the pack capacity are never live and keep no row)
        float* row = &rows[threadIdx.x * kRowPad];
        const int p4 = live ? (int)gld(d.pos4 + i) : (0 | (1 << 3) | (2 << 6) | (3 << 9));
        const int jd = d.jac_dtype;          // uniform: one branch for the whole row
        if (jd != 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    Jw[k][c] = keep_jac(Jw[k][c], jd);
                    Jt[k][c] = keep_jac(Jt[k][c], jd);
                }
        }
        int used = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int pos = (p4 >> (3 * k)) & 7;
            used |= 1 << pos;
            float* o = row + pos * 6;
            o[0] = Jw[k][0]; o[1] = Jw[k][1]; o[2] = Jw[k][2];
            o[3] = Jt[k][0]; o[4] = Jt[k][1]; o[5] = Jt[k][2];
        }
        // the segment's fifth node position, if the surfel does not touch it
#pragma unroll
        for (int pos = 0; pos < 5; ++pos)
            if (!(used & (1 << pos))) {
#pragma unroll
                for (int c = 0; c < 6; ++c) row[pos * 6 + c] = 0.f;
            }
        row[30] = r;
    }
    if (threadIdx.x == kCorrBlock - 1) {
        // read (as column 31, whose products are dropped) past the last row
#pragma unroll
        for (int c = 0; c < 8; ++c) rows[kCorrPack * kRowPad + c] = 0.f;
    }
    if (live && capture) {
        capture_live(d, org, wp);
        if (matched) d.dbg_corr[pix] = org;
    }
    double e = block_sum((double)r * (double)r, sh);   // (synchronises the rows too)
    int cnt = wave_sumi(matched ? 1 : 0);
    if ((threadIdx.x % kWave) == 0) shi[threadIdx.x / kWave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int c = 0;
        for (int q = 0; q < (int)(blockDim.x / kWave); ++q) c += shi[q];
        gst(d.part_e + at.tile, e);
        gst(d.part_n + at.tile, c);
    }
    if (capture) {
        // the wave's rows as whole 128-byte lines, two rows per store
        const int base = wave * kWave;
        float* dst = d.J + (size_t)(p0 + base) * 32;
        const int nrow = min(kWave, p1 - p0 - base);
        for (int q = 0; q < kWave / 2; ++q) {
            const int rr = 2 * q + (lane >> 5), c = lane & 31;
            if (rr < nrow) dst[rr * 32 + c] = c < 31 ? rows[(base + rr) * kRowPad + c] : 0.f;
        }
    }
    // segment Gram matrices, one wave per segment
    segment_grams(d, rows, stage4[wave], at.tile, p0, nullptr);
}

// ---------------------------------------------------------------------------
// Rigid alignment before the non-rigid steps (Sec. 7: a rigid alignment as in
// KinectFusion precedes the non-rigid estimation): projective point-to-plane
// ICP of one transform T = (R_c, t_c) applied after the warp field.
//   rigid_warp   y_i = R_c v'_i + t_c into the index map
//   rigid_sys    correspondence on y_i, r_i = N^T (y_i - V), J_i = (y_i x N, N);
//                per tile the sums of J J^T (upper 21), J r, r^2 and the count
//   rigid_solve  (sum J J^T + mu I) xi = -sum J r in FP64 (one workgroup per
//                stream, fixed summation order), T <- (Exp(w) R_c, Exp(w) t_c + tau);
//                every workgroup also resets the index map
//   rigid_compose  T_k <- T o T_k for every node
// ---------------------------------------------------------------------------
__device__ __forceinline__ float3 rigid_apply(const float* __restrict__ T, float3 v) {
    return make_float3(((T[0] * v.x + T[1] * v.y) + T[2] * v.z) + T[9],
                       ((T[3] * v.x + T[4] * v.y) + T[5] * v.z) + T[10],
                       ((T[6] * v.x + T[7] * v.y) + T[8] * v.z) + T[11]);
}
__device__ __forceinline__ float3 rigid_rotate(const float* __restrict__ T, float3 v) {
    return make_float3((T[0] * v.x + T[1] * v.y) + T[2] * v.z, (T[3] * v.x + T[4] * v.y) + T[5] * v.z,
                       (T[6] * v.x + T[7] * v.y) + T[8] * v.z);
}

__global__ void __launch_bounds__(kWarpBlock) k_rigid_warp(Batch b) {
    const Where at = locate(b);
    const FrameDesc d = *b.d[at.s];
    const int i = at.tile * kWarpBlock + threadIdx.x;
    if (i >= d.ns || !visible(d, i)) return;
    float T[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) T[q] = d.rig[q];
    const float3 v = make_float3(d.px[i], d.py[i], d.pz[i]);
    const Warp wp = warp_surfel(d.idx[i], d.w[i], v, make_float3(0.f, 0.f, 0.f), d.dq);
    if (!wp.ok) return;
    const float3 y = rigid_apply(T, wp.v);
    int ux, uy;
    if (!project(d.cam, y, ux, uy)) return;
    atomicMin(&d.zbuf[uy * d.cam.W + ux], zkey(y.z, d.orig[i]));
}

__global__ void __launch_bounds__(256) k_rigid_sys(Batch b) {
    __shared__ double ws[4][kRigidSums];
    const Where at = locate(b);
    const FrameDesc d = *b.d[at.s];
    float T[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) T[q] = d.rig[q];
    double acc[kRigidSums];
#pragma unroll
    for (int q = 0; q < kRigidSums; ++q) acc[q] = 0.0;
    for (int u = 0; u < kRigidSurfels / 256; ++u) {
        const int i = at.tile * kRigidSurfels + u * 256 + threadIdx.x;
        if (i >= d.ns) break;
        const float3 v = make_float3(d.px[i], d.py[i], d.pz[i]);
        const float3 n = make_float3(d.nx[i], d.ny[i], d.nz[i]);
        const Warp wp = warp_surfel(d.idx[i], d.w[i], v, n, d.dq);
        if (!wp.ok) continue;
        const float3 y = rigid_apply(T, wp.v);
        const float3 ny = rigid_rotate(T, wp.n);
        int ux, uy;
        if (!project(d.cam, y, ux, uy)) continue;
        const int pix = uy * d.cam.W + ux;
        if (d.zbuf[pix] != zkey(y.z, d.orig[i])) continue;
        const float4 nm = d.nmap[pix];
        if (!(nm.w > 0.f)) continue;
        const float3 V = backproject(d.cam, ux, uy, nm.w);
        const float3 dv = sub3(y, V);
        const float d2 = (dv.x * dv.x + dv.y * dv.y) + dv.z * dv.z;
        const float3 N = make_float3(nm.x, nm.y, nm.z);
        if (!(d2 < d.dist2 && dot3(ny, N) > d.cosn)) continue;
        const double r = (double)dot3(N, dv);
        const float3 c = cross3(y, N);
        const double J[6] = {c.x, c.y, c.z, N.x, N.y, N.z};
        int q = 0;
#pragma unroll
        for (int a = 0; a < 6; ++a)
#pragma unroll
            for (int bb = a; bb < 6; ++bb) acc[q++] += J[a] * J[bb];
#pragma unroll
        for (int a = 0; a < 6; ++a) acc[21 + a] += J[a] * r;
        acc[27] += r * r;
        acc[28] += 1.0;
    }
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < kRigidSums; ++q) {
        const double v = wave_sum(acc[q]);
        if (lane == 0) ws[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < kRigidSums) {
        double t = 0.0;
        for (int w = 0; w < 4; ++w) t += ws[w][threadIdx.x];
        d.rig_part[(size_t)at.tile * kRigidSums + threadIdx.x] = t;
    }
}

__global__ void __launch_bounds__(kNodeBlock) k_rigid_solve(Batch b) {
    __shared__ double part[8][kRigidSums];
    __shared__ double tot[kRigidSums];
    const Where at = locate(b);
    const FrameDesc d = *b.d[at.s];
    const int gid = at.tile * kNodeBlock + threadIdx.x;
    if (gid < d.npx) d.zbuf[gid] = ~0ull;     // index map of the next step
    if (at.tile != 0) return;
    // sums over tiles: quantity q, tiles congruent to l mod 8, then the 8 in order
    const int ntiles = cdiv(d.ns, kRigidSurfels);
    if (threadIdx.x < 8 * kRigidSums) {
        const int q = threadIdx.x % kRigidSums, l = threadIdx.x / kRigidSums;
        double v = 0.0;
        for (int t = l; t < ntiles; t += 8) v += d.rig_part[(size_t)t * kRigidSums + q];
        part[l][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < kRigidSums) {
        double v = 0.0;
        for (int l = 0; l < 8; ++l) v += part[l][threadIdx.x];
        tot[threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int step = b.it[at.s];
    double A[6][6], g[6];
    int q = 0;
    for (int a = 0; a < 6; ++a)
        for (int c = a; c < 6; ++c) {
            A[a][c] = tot[q];
            A[c][a] = tot[q];
            ++q;
        }
    for (int a = 0; a < 6; ++a) {
        A[a][a] += (double)d.mu;
        g[a] = tot[21 + a];
    }
    d.rig_stats[step].e = tot[27];
    d.rig_stats[step].n = (int)tot[28];
    // Cholesky A = L L^T, then xi = -A^-1 g
    double L[6][6];
    bool ok = true;
    for (int a = 0; a < 6; ++a) {
        for (int c = 0; c <= a; ++c) {
            double s = A[a][c];
            for (int k = 0; k < c; ++k) s -= L[a][k] * L[c][k];
            if (a == c) {
                ok = ok && (s > 0.0);
                L[a][a] = sqrt(s > 0.0 ? s : 1.0);
            } else {
                L[a][c] = s / L[c][c];
            }
        }
    }
    double y[6], xi[6];
    for (int a = 0; a < 6; ++a) {
        double s = -g[a];
        for (int k = 0; k < a; ++k) s -= L[a][k] * y[k];
        y[a] = s / L[a][a];
    }
    for (int a = 5; a >= 0; --a) {
        double s = y[a];
        for (int k = a + 1; k < 6; ++k) s -= L[k][a] * xi[k];
        xi[a] = s / L[a][a];
    }
    for (int a = 0; a < 6; ++a) ok = ok && (fabs(xi[a]) < INFINITY);
    if (!ok) {
        atomicOr(d.flags, 8);
        return;
    }
    // Exp(w) by Rodrigues, T <- (E R_c, E t_c + tau)
    const double th = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
    double E[9];
    {
        const double kx = xi[0], ky = xi[1], kz = xi[2];
        double s1, c1;
        if (th < 1e-12) {
            s1 = 1.0;            // sin(th) / th
            c1 = 0.5;            // (1 - cos(th)) / th^2
        } else {
            s1 = sin(th) / th;
            c1 = (1.0 - cos(th)) / (th * th);
        }
        E[0] = 1.0 - c1 * (ky * ky + kz * kz); E[1] = c1 * kx * ky - s1 * kz;  E[2] = c1 * kx * kz + s1 * ky;
        E[3] = c1 * kx * ky + s1 * kz;  E[4] = 1.0 - c1 * (kx * kx + kz * kz); E[5] = c1 * ky * kz - s1 * kx;
        E[6] = c1 * kx * kz - s1 * ky;  E[7] = c1 * ky * kz + s1 * kx;  E[8] = 1.0 - c1 * (kx * kx + ky * ky);
    }
    double Rn[9], tn[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c)
            Rn[3 * r + c] = E[3 * r] * d.rig64[c] + E[3 * r + 1] * d.rig64[3 + c] + E[3 * r + 2] * d.rig64[6 + c];
        tn[r] = E[3 * r] * d.rig64[9] + E[3 * r + 1] * d.rig64[10] + E[3 * r + 2] * d.rig64[11] + xi[3 + r];
    }
    for (int k = 0; k < 9; ++k) {
        d.rig64[k] = Rn[k];
        d.rig[k] = (float)Rn[k];
    }
    for (int k = 0; k < 3; ++k) {
        d.rig64[9 + k] = tn[k];
        d.rig[9 + k] = (float)tn[k];
    }
}

// Unit quaternion (w >= 0) of a rotation matrix, FP64.
__device__ __forceinline__ void quat_of(const double* m, double& qw, double& qx, double& qy, double& qz) {
    const double R00 = m[0], R01 = m[1], R02 = m[2], R10 = m[3], R11 = m[4], R12 = m[5], R20 = m[6],
                 R21 = m[7], R22 = m[8];
    const double tr = R00 + R11 + R22;
    if (tr >= R00 && tr >= R11 && tr >= R22) {
        const double s = 2.0 * sqrt(fmax(1.0 + tr, 0.0));
        qw = 0.25 * s; qx = (R21 - R12) / s; qy = (R02 - R20) / s; qz = (R10 - R01) / s;
    } else if (R00 >= R11 && R00 >= R22) {
        const double s = 2.0 * sqrt(fmax(1.0 + R00 - R11 - R22, 0.0));
        qw = (R21 - R12) / s; qx = 0.25 * s; qy = (R01 + R10) / s; qz = (R02 + R20) / s;
    } else if (R11 >= R22) {
        const double s = 2.0 * sqrt(fmax(1.0 - R00 + R11 - R22, 0.0));
        qw = (R02 - R20) / s; qx = (R01 + R10) / s; qy = 0.25 * s; qz = (R12 + R21) / s;
    } else {
        const double s = 2.0 * sqrt(fmax(1.0 - R00 - R11 + R22, 0.0));
        qw = (R10 - R01) / s; qx = (R02 + R20) / s; qy = (R12 + R21) / s; qz = 0.25 * s;
    }
    const double nq = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    const double sg = qw < 0 ? -1.0 : 1.0;
    qw *= sg / nq; qx *= sg / nq; qy *= sg / nq; qz *= sg / nq;
}

__global__ void __launch_bounds__(kNodeBlock) k_rigid_compose(Batch b) {
    const Where at = locate(b);
    const FrameDesc d = *b.d[at.s];
    const int k = at.tile * kNodeBlock + threadIdx.x;
    if (k >= d.nn) return;
    double cw, cx, cy, cz;
    quat_of(d.rig64, cw, cx, cy, cz);
    const float4 q = d.rq[k];
    const double kw = q.x, kx = q.y, ky = q.z, kz = q.w;
    // q_c (x) q_k, renormalised, w >= 0
    double rw = cw * kw - cx * kx - cy * ky - cz * kz;
    double rx = cw * kx + cx * kw + cy * kz - cz * ky;
    double ry = cw * ky - cx * kz + cy * kw + cz * kx;
    double rz = cw * kz + cx * ky - cy * kx + cz * kw;
    const double nr = sqrt(rw * rw + rx * rx + ry * ry + rz * rz) * (rw < 0 ? -1.0 : 1.0);
    rw /= nr; rx /= nr; ry /= nr; rz /= nr;
    const float4 t4 = d.tt[k];
    const double* m = d.rig64;
    const double tx = m[0] * t4.x + m[1] * t4.y + m[2] * t4.z + m[9];
    const double ty = m[3] * t4.x + m[4] * t4.y + m[5] * t4.z + m[10];
    const double tz = m[6] * t4.x + m[7] * t4.y + m[8] * t4.z + m[11];
    const Q4 r = Q4{(float)rw, (float)rx, (float)ry, (float)rz};
    const float3 t = make_float3((float)tx, (float)ty, (float)tz);
    d.rq[k] = f4(r);
    d.tt[k] = make_float4(t.x, t.y, t.z, 0.f);
    node_tables(d.pref[k], r, t, d.dq, d.cl, k);
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
void launch_frame_stage(int stage, const Batch& b, const DepthIn* depth, hipStream_t st) {
    const int grid = b.off[b.n];
    if (grid <= 0) return;
    switch (stage) {
        case kStDepth: hipLaunchKernelGGL(k_depth_prep, dim3(grid), dim3(256), 0, st, b, *depth); break;
        case kStWarp:
            if (b.splat) hipLaunchKernelGGL(k_warp_zbuf<true>, dim3(grid), dim3(kWarpBlock), 0, st, b);
            else hipLaunchKernelGGL(k_warp_zbuf<false>, dim3(grid), dim3(kWarpBlock), 0, st, b);
            break;
        case kStCorr:
            if (b.splat) hipLaunchKernelGGL(k_corr_gram<true>, dim3(grid), dim3(kCorrBlock), 0, st, b);
            else hipLaunchKernelGGL(k_corr_gram<false>, dim3(grid), dim3(kCorrBlock), 0, st, b);
            break;
        case kStRigidWarp: hipLaunchKernelGGL(k_rigid_warp, dim3(grid), dim3(kWarpBlock), 0, st, b); break;
        case kStRigidSys: hipLaunchKernelGGL(k_rigid_sys, dim3(grid), dim3(256), 0, st, b); break;
        case kStRigidSolve: hipLaunchKernelGGL(k_rigid_solve, dim3(grid), dim3(kNodeBlock), 0, st, b); break;
        case kStRigidCompose: hipLaunchKernelGGL(k_rigid_compose, dim3(grid), dim3(kNodeBlock), 0, st, b); break;
        default: break;
    }
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

__global__ void k_map_ids(int* __restrict__ p, int n, const int* __restrict__ map) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = map[p[i]];
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

void launch_map_ids(int* p, int n, const int* map, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_map_ids, dim3((n + 255) / 256), dim3(256), 0, st, p, n, map);
}

void launch_tables_from_state(int nn, const float4* pref, const float4* rq, const float4* tt, float4* dq, float4* cl,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_tables_from_state, dim3((nn + 255) / 256), dim3(256), 0, st, nn, pref, rq, tt, dq, cl);
}

}  // namespace swgn
