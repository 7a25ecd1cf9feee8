// C ABI of the swgn library: stream objects, device memory, the setup
// pipeline and the per-frame Gauss-Newton driver for one stream or a batch.
//
// Memory of a stream is in two parts:
//   resident   surfels, skinning, node state, node graph, block pattern and
//              work lists: allocated by sw_set_node_graph, kept for the
//              stream's life;
//   workspace  everything a frame in flight needs (depth copy, normal and
//              index maps, Jacobian rows, segment Grams, blocks, PCG vectors,
//              partials, statistics): one contiguous carve-out whose size
//              follows from the stream's shapes.
// Both are described to the kernels by the stream's FrameDesc, a device copy
// of which is rewritten whenever a pointer in it changes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "runtime_internal.h"
#include "segments.h"
#include "swgn_setup.h"
#include "swgn_fusion.h"
#include "swgn.h"
#include "swgn_frame.h"
#include "swgn_impl.h"
#include "swgn_launch.h"

using namespace swgn;
using namespace swgn::rt;

namespace swgn {
namespace rt {

void* Arena::raw(size_t bytes) {
    constexpr size_t kFirstChunk = (size_t)4 << 20, kMaxChunk = (size_t)256 << 20;
    bytes = ((bytes == 0 ? 1 : bytes) + 255) & ~size_t(255);
    for (; cur_ < chunks_.size(); ++cur_) {
        Chunk& c = chunks_[cur_];
        if (c.size - c.used >= bytes) {
            char* p = c.base + c.used;
            c.used += bytes;
            bytes_ += bytes;
            return p;
        }
    }
    const size_t grow = chunks_.empty() ? kFirstChunk : std::min(kMaxChunk, 2 * chunks_.back().size);
    const size_t size = std::max(bytes, grow);
    void* p = nullptr;
    SWGN_HIP(hipMalloc(&p, size));
    chunks_.push_back(Chunk{static_cast<char*>(p), size, bytes});
    cur_ = chunks_.size() - 1;
    bytes_ += bytes;
    return p;
}

void Arena::release() {
    for (const Chunk& c : chunks_) (void)hipFree(c.base);
    chunks_.clear();
    cur_ = 0;
    bytes_ = 0;
}

void Arena::reset() {
    for (Chunk& c : chunks_) c.used = 0;
    cur_ = 0;
    bytes_ = 0;
}

void Executor::drop_graph() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    graph_exec = nullptr;
    graph_key.clear();
}

Executor::~Executor() {
    drop_graph();
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    if (stats_host) (void)hipHostFree(stats_host);
    if (stats_dev) (void)hipFree(stats_dev);
    if (own_stream && st) (void)hipStreamDestroy(st);
}

void Executor::init(void* hip_stream) {
    if (hip_stream) {
        st = static_cast<hipStream_t>(hip_stream);
    } else {
        SWGN_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        own_stream = true;
    }
    SWGN_HIP(hipMalloc(reinterpret_cast<void**>(&stats_dev), (size_t)kStatsOutBytes * kMaxBatch));
    SWGN_HIP(hipHostMalloc(&stats_host, (size_t)kStatsOutBytes * kMaxBatch, hipHostMallocDefault));
}

int Executor::variant_of(int stage, int64_t rows) const {
    const auto it = tuned.find(bucket);
    if (it != tuned.end()) return it->second[stage];
    // untuned: the wide geometries only when the launch still has two
    // workgroups per CU with them
    const bool wide = (stage == kStSpmv && rows >= 256 * 2 * kSpmvRows) ||
                      (stage == kStUpdate && rows >= 256 * 2 * 2 * kSolveNodes);
    // fused PCG steps while the product launch is too small to fill the chip
    const bool fused = stage == kStSpmv && rows <= kFusedRows;
    // the PCG's tiles XCD-contiguous: with nodes in spatial order, an XCD's
    // rows then share their columns (measured: a faster fused step; the fold
    // and the initialisation were slower so)
    const bool xcd = stage == kStSpmv || stage == kStUpdate || stage == kStPcgStep;
    return (wide ? kVarWide : 0) | (fused ? kVarFused : 0) | (xcd ? kVarXcd : 0);
}

// Shape bucket of a batch: the stream count and the powers of two of its total
// surfels and nodes. Tuned choices are kept per bucket.
uint64_t shape_bucket(const std::vector<sw_stream>& ss) {
    int64_t ns = 0, nn = 0;
    for (sw_stream s : ss) {
        ns += s->h.ns;
        nn += s->h.nn;
    }
    auto lg = [](int64_t v) {
        uint64_t b = 0;
        while (((int64_t)1 << b) < v) ++b;
        return b;
    };
    return ((uint64_t)ss.size() << 16) | (lg(ns) << 8) | lg(nn);
}

hipEvent_t Executor::event(size_t i) {
    while (events.size() <= i) {
        hipEvent_t e;
        SWGN_HIP(hipEventCreate(&e));
        events.push_back(e);
    }
    return events[i];
}

// Carves the workspace of a stream with shapes h from base (or, with base
// null, only sums its size). Every piece is 256-byte aligned.
size_t carve_workspace(FrameDesc& h, char* base) {
    size_t off = 0;
    auto take = [&](auto*& p, size_t bytes) {
        using T = std::remove_reference_t<decltype(*p)>;
        p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += (bytes + 255) & ~size_t(255);
    };
    const size_t npx = (size_t)h.npx, nn = (size_t)h.nn;
    const size_t nsol = (size_t)solve_parts(h), nspm = (size_t)spmv_parts(h), ncor = (size_t)corr_tiles(h);
    take(h.depth, 4 * npx);
    take(h.nmap, 16 * npx);
    take(h.zbuf, 8 * npx);
    take(h.flags, 16);
    take(h.stats, sizeof(IterStats) * kMaxIters);
    take(h.rq_bak, 16 * nn);
    take(h.tt_bak, 16 * nn);
    take(h.part, 4 * (size_t)std::max<int64_t>(1, h.part_floats));
    take(h.H, 144 * (size_t)h.nb);
    take(h.Hf, 144 * nn * (size_t)h.ell_w);
    take(h.g, 24 * nn);
    take(h.ereg, 4 * nn);
    take(h.Minv, 288 * nn);
    take(h.part_e, 8 * ncor);
    take(h.part_n, 4 * ncor);
    take(h.x, 24 * nn);
    for (int q = 0; q < 2; ++q) {
        auto half = [q](auto& pp) -> auto& { return q ? pp.b1 : pp.b0; };
        take(half(h.r), 24 * nn);
        take(half(h.z), 24 * nn);
        take(half(h.p), 24 * nn);
        take(half(h.u), 24 * nn);
        take(half(h.v), 24 * nn);
        take(half(h.part_rho), 8 * nsol);
        take(half(h.part_rr), 8 * nsol);
        take(half(h.part_c), 3 * 8 * nspm);
    }
    take(h.sc, 16);
    take(h.rig, 12 * 4);
    take(h.rig64, 12 * 8);
    take(h.rig_part, 8 * (size_t)kRigidSums * (size_t)cdiv(h.ns, kRigidSurfels));
    take(h.rig_stats, sizeof(RigidStats) * kMaxIters);
    return off;
}

}  // namespace rt
}  // namespace swgn

namespace {

bool finite(float v) { return std::isfinite(v); }

int pow2_at_least(int64_t n, int lo) {
    int64_t p = lo;
    while (p < n) p <<= 1;
    return (int)p;
}

sw_status check_config(const sw_config* c, std::string& why) {
    if (!c) { why = "config is NULL"; return SW_EINVAL; }
    if (c->width <= 0 || c->height <= 0 || c->width > 16384 || c->height > 16384) {
        why = "image size out of range"; return SW_EINVAL;
    }
    if (!(finite(c->fx) && finite(c->fy) && c->fx > 0 && c->fy > 0 && finite(c->cx) && finite(c->cy))) {
        why = "intrinsics must be finite with positive focal lengths"; return SW_EINVAL;
    }
    if (c->gn_iters < 0 || c->gn_iters > kMaxIters) { why = "gn_iters must be in [0, 16]"; return SW_EINVAL; }
    if (c->pcg_iters < 0 || c->pcg_iters > kMaxPcg) { why = "pcg_iters must be in [0, 4096]"; return SW_EINVAL; }
    if (!(finite(c->lambda_reg) && c->lambda_reg >= 0)) { why = "lambda_reg must be >= 0"; return SW_EINVAL; }
    if (!(finite(c->node_sigma) && c->node_sigma > 0)) { why = "node_sigma must be > 0"; return SW_EINVAL; }
    if (!(finite(c->corr_dist) && c->corr_dist > 0)) { why = "corr_dist must be > 0"; return SW_EINVAL; }
    if (!(finite(c->corr_normal) && c->corr_normal >= -1 && c->corr_normal <= 1)) {
        why = "corr_normal must be in [-1, 1]"; return SW_EINVAL;
    }
    if (!(finite(c->edge_gate) && c->edge_gate >= 0)) { why = "edge_gate must be >= 0"; return SW_EINVAL; }
    if (!(finite(c->damping) && c->damping >= 0)) { why = "damping must be >= 0"; return SW_EINVAL; }
    if (c->jac_dtype < 0 || c->jac_dtype > 2) { why = "jac_dtype must be 0 (fp32), 1 (bf16) or 2 (fp16)"; return SW_EINVAL; }
    if (c->dot_fp64 != 1) { why = "dot_fp64: PCG dot products accumulate in fp64 (1)"; return SW_EINVAL; }
    if (c->debug_iter < -1 || c->debug_iter >= kMaxIters) { why = "debug_iter out of range"; return SW_EINVAL; }
    if (c->stage_timing != 0 && c->stage_timing != 1) { why = "stage_timing must be 0 or 1"; return SW_EINVAL; }
    if (c->rigid_iters < 0 || c->rigid_iters > kMaxIters) { why = "rigid_iters must be in [0, 16]"; return SW_EINVAL; }
    if (c->visibility != 0 && c->visibility != 1) { why = "visibility must be 0 or 1"; return SW_EINVAL; }
    if (!finite(c->stable_conf)) { why = "stable_conf must be finite"; return SW_EINVAL; }
    if (c->recent_frames < -1) { why = "recent_frames must be >= -1"; return SW_EINVAL; }
    if (!(finite(c->fusion_dist) && c->fusion_dist > 0)) { why = "fusion_dist must be > 0"; return SW_EINVAL; }
    if (!(finite(c->fusion_normal) && c->fusion_normal >= -1 && c->fusion_normal <= 1)) {
        why = "fusion_normal must be in [-1, 1]"; return SW_EINVAL;
    }
    if (!(finite(c->warp_eps) && c->warp_eps > 0 && c->warp_eps < 1)) { why = "warp_eps must be in (0, 1)"; return SW_EINVAL; }
    if (!(finite(c->append_nn) && c->append_nn >= 0)) { why = "append_nn must be >= 0"; return SW_EINVAL; }
    if (c->t_low_confid < 0) { why = "t_low_confid must be >= 0"; return SW_EINVAL; }
    if (c->splat != 0 && c->splat != 1) { why = "splat must be 0 or 1"; return SW_EINVAL; }
    return SW_OK;
}

// H2D (host) or D2D (device) copy onto the stream.
void copy_in(void* dst, const void* src, size_t bytes, int32_t on_device, hipStream_t st) {
    SWGN_HIP(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
}

template <class T>
T read_scalar(const T* dptr, hipStream_t st) {
    T v;
    SWGN_HIP(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, st));
    SWGN_HIP(hipStreamSynchronize(st));
    return v;
}

// Writes the stream's descriptor to its device copy.
void publish_desc(sw_stream s) {
    *s->h_pinned = s->h;
    SWGN_HIP(hipMemcpyAsync(s->d_desc, s->h_pinned, sizeof(FrameDesc), hipMemcpyHostToDevice, s->exec.st));
    SWGN_HIP(hipStreamSynchronize(s->exec.st));
}

// Segments, packs and the block fold's entries (once per node set, on the
// device).
//
// A segment is a run of consecutive surfels (sorted by node set), at most
// kCorrPack long, whose nodes together number at most 5: its Gram matrix
// [J | r]^T [J | r] (30 Jacobian columns, node blocks by position in the
// segment's ascending node list, r in column 30) fits one 32x32 MFMA tile.
// It keeps the 6x6 sub-blocks of the node pairs that share a surfel (bit
// first(pa) + pb - pa of its 15-bit mask, pa <= pb), then J^T r (30) and
// r^T r: 36 x pairs + 32 floats from offset seg_off. A pack is a greedy run
// of whole segments with at most kCorrPack surfels. Each block's entries
// list the float offsets of its sub-blocks (and, for a diagonal block, of the
// matching J^T r piece) in segment order.
// The greedy cuts are successor chains walked on the device (segwalk.hip);
// the host reads back three sizes (segments; Gram floats, entries and packs;
// the consistency flag) to size the resident arrays.
void build_segments(sw_stream s, FrameDesc& h, const uint64_t* key, const int* set_start, const int* run_pos,
                    int nsets, const int4* sidx, const int* row_ptr, const int* col_idx, Arena& G, Arena& tmp) {
    hipStream_t st = s->exec.st;
    const int ns = h.ns, nb = h.nb;
    if (kCorrPack > chain_max_hop()) throw HipFail{hipErrorInvalidValue, "segment layout: pack size above the chain hop"};
    uint64_t* d_keys = tmp.alloc<uint64_t>(std::max(1, nsets));
    launch_set_keys(nsets, key, set_start, d_keys, st);
    int* d_bad = tmp.alloc<int>(1);
    int* d_cnt = tmp.alloc<int>(2);
    unsigned long long* d_units = tmp.alloc<unsigned long long>(1);
    launch_fill_i32(d_bad, 1, 0, st);
    launch_fill_i32(reinterpret_cast<int*>(d_units), 2, 0, st);
    int* work = tmp.alloc<int>(chain_work_ints(ns, kCorrPack));
    int* scan_tmp = tmp.alloc<int>(scan_tmp_size(std::max(ns, nb) + 16));

    // segment cuts
    int* nxt = tmp.alloc<int>(ns);
    int* cuts = tmp.alloc<int>(ns);
    launch_seg_next(ns, nsets, d_keys, set_start, run_pos, kCorrPack, nxt, st);
    chain_from_zero(nxt, ns, kCorrPack, cuts, d_cnt, work, d_bad, st);
    int cut[2] = {0, 0};                       // segments, flag
    SWGN_HIP(hipMemcpyAsync(&cut[0], d_cnt, sizeof(int), hipMemcpyDeviceToHost, st));
    SWGN_HIP(hipMemcpyAsync(&cut[1], d_bad, sizeof(int), hipMemcpyDeviceToHost, st));
    SWGN_HIP(hipStreamSynchronize(st));
    const int nseg = cut[0];
    if (cut[1] != 0 || nseg < 1 || nseg > ns)
        throw HipFail{hipErrorInvalidValue, "segment layout: the segment cut is inconsistent"};
    int* d_seg = G.alloc<int>(nseg + 1);
    SWGN_HIP(hipMemcpyAsync(d_seg, cuts, sizeof(int) * nseg, hipMemcpyDeviceToDevice, st));
    launch_fill_i32(d_seg + nseg, 1, ns, st);

    // per segment: nodes, pair mask, output offsets, entry bases; packs
    int* d_nodes = tmp.alloc<int>(5 * (size_t)nseg);
    uint16_t* d_mask = G.alloc<uint16_t>(nseg);
    int* units = tmp.alloc<int>(nseg);
    int* npairs = tmp.alloc<int>(nseg);
    launch_seg_info(nseg, d_seg, run_pos, d_keys, d_nodes, d_mask, units, npairs, d_units, d_bad, st);
    int* off_units = tmp.alloc<int>(nseg + 1);
    int* ebase = tmp.alloc<int>(nseg + 1);
    exclusive_scan(units, off_units, nseg, scan_tmp, st);
    exclusive_scan(npairs, ebase, nseg, scan_tmp, st);
    int* pnext = tmp.alloc<int>(nseg);
    int* pcuts = tmp.alloc<int>(nseg);
    launch_pack_next(nseg, d_seg, kCorrPack, pnext, st);
    chain_from_zero(pnext, nseg, kCorrPack, pcuts, d_cnt + 1, work, d_bad, st);
    unsigned long long total_units = 0;
    int sizes[3] = {0, 0, 0};                  // entries, packs, flag
    SWGN_HIP(hipMemcpyAsync(&total_units, d_units, sizeof(total_units), hipMemcpyDeviceToHost, st));
    SWGN_HIP(hipMemcpyAsync(&sizes[0], ebase + nseg, sizeof(int), hipMemcpyDeviceToHost, st));
    SWGN_HIP(hipMemcpyAsync(&sizes[1], d_cnt + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    SWGN_HIP(hipMemcpyAsync(&sizes[2], d_bad, sizeof(int), hipMemcpyDeviceToHost, st));
    SWGN_HIP(hipStreamSynchronize(st));
    if (sizes[2] != 0) throw HipFail{hipErrorInvalidValue, "segment layout: a segment has more than 5 nodes"};
    if (total_units >= (1ull << 30)) throw HipFail{hipErrorInvalidValue, "segment Gram storage exceeds 2^32 floats"};
    const int ne = sizes[0], npack = sizes[1];
    if (ne < 1 || npack < 1 || npack > nseg)
        throw HipFail{hipErrorInvalidValue, "segment layout: the pack cut is inconsistent"};
    uint32_t* d_off = G.alloc<uint32_t>(nseg + 1);
    launch_seg_off(nseg, off_units, d_off, st);

    // the fold's entries, sorted by block (stable in segment order)
    const int npad = pow2_at_least(ne, 1024);
    uint64_t* ekey = tmp.alloc<uint64_t>(npad);
    uint32_t* eval = tmp.alloc<uint32_t>(npad);
    uint32_t* esub = tmp.alloc<uint32_t>(ne);
    uint32_t* egrad = tmp.alloc<uint32_t>(ne);
    int* bcount = tmp.alloc<int>(nb);
    launch_fill_i32(bcount, nb, 0, st);
    launch_seg_entries(nseg, nb, npad, d_nodes, d_mask, d_off, ebase, ne, row_ptr, col_idx, ekey, eval, esub, egrad,
                       bcount, d_bad, st);
    sort_pairs(ekey, eval, npad, st);
    int* d_ep = G.alloc<int>(nb + 1);
    exclusive_scan(bcount, d_ep, nb, scan_tmp, st);
    uint32_t* d_es = G.alloc<uint32_t>(ne);
    uint32_t* d_eg = G.alloc<uint32_t>(ne);
    launch_ent_gather(ne, eval, esub, egrad, d_es, d_eg, st);

    // packs
    int* d_pg = G.alloc<int>(npack + 1);
    int* d_ps = G.alloc<int>(npack + 1);
    SWGN_HIP(hipMemcpyAsync(d_pg, pcuts, sizeof(int) * npack, hipMemcpyDeviceToDevice, st));
    launch_pack_arrays(npack, nseg, ns, d_seg, d_pg, d_ps, st);

    // each surfel's node positions in its segment
    uint16_t* d_pos4 = G.alloc<uint16_t>(ns);
    launch_seg_pos4(ns, nseg, d_seg, d_nodes, sidx, d_pos4, d_bad, st);
    SWGN_HIP(hipGetLastError());
    if (read_scalar(d_bad, st) != 0)
        throw HipFail{hipErrorInvalidValue, "segment layout: a block or a surfel's node is missing from its segment"};
    h.nseg = nseg;
    h.npack = npack;
    h.part_floats = 4 * (int64_t)total_units;
    h.seg_start = d_seg;
    h.pos4 = d_pos4;
    h.seg_mask = d_mask;
    h.seg_off = d_off;
    h.pack_start = d_ps;
    h.pack_seg = d_pg;
    h.ent_ptr = d_ep;
    h.ent_sub = d_es;
    h.ent_grad = d_eg;
    s->nent = ne;
}

// The library's node order: ascending Morton code of the reference positions
// (10 bits per axis over their bounding box), ties by the caller's index.
// Consecutive nodes are then near each other, and so are a block row's
// columns (its graph neighbours and the nodes sharing its surfels).
static std::vector<int> morton_order(const std::vector<float>& pos, int nn) {
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int k = 0; k < nn; ++k)
        for (int a = 0; a < 3; ++a) {
            const float v = pos[3 * k + a];
            if (std::isfinite(v)) { lo[a] = std::min(lo[a], v); hi[a] = std::max(hi[a], v); }
        }
    auto spread = [](uint32_t v) {      // 10 bits -> every third bit
        v &= 1023u;
        v = (v | (v << 16)) & 0x030000FFu;
        v = (v | (v << 8)) & 0x0300F00Fu;
        v = (v | (v << 4)) & 0x030C30C3u;
        v = (v | (v << 2)) & 0x09249249u;
        return v;
    };
    std::vector<std::pair<uint32_t, int>> key((size_t)nn);
    for (int k = 0; k < nn; ++k) {
        uint32_t q[3];
        for (int a = 0; a < 3; ++a) {
            const float ext = hi[a] - lo[a];
            const float v = pos[3 * k + a];
            const float t = (ext > 0.f && std::isfinite(v)) ? (v - lo[a]) / ext : 0.f;
            q[a] = (uint32_t)std::min(1023.f, std::max(0.f, t * 1023.f));
        }
        key[(size_t)k] = {spread(q[0]) | (spread(q[1]) << 1) | (spread(q[2]) << 2), k};
    }
    std::sort(key.begin(), key.end());
    std::vector<int> perm((size_t)nn);
    for (int k = 0; k < nn; ++k) perm[(size_t)k] = key[(size_t)k].second;
    return perm;
}

// keep_order: node_pos is in the library's order and the numbering stays (a
// rebuild after a geometry update; the node state keep_rq / keep_tt is in
// that order too).
void build_graph(sw_stream s, int nn, const float* node_pos, const float* node_se3, int32_t on_device,
                 const float4* keep_rq, const float4* keep_tt, bool keep_order) {
    hipStream_t st = s->exec.st;
    // the node-set arrays and temporaries reuse their device memory: no work
    // of the device may still use it
    SWGN_HIP(hipDeviceSynchronize());
    s->graph_mem.reset();
    s->ws_mem.release();
    s->graph_set = false;
    s->captured = false;
    ++s->generation;
    Arena& tmp = s->setup_mem;
    tmp.reset();
    Arena& G = s->graph_mem;
    const int ns = (int)s->ns;
    FrameDesc h{};
    h.ns = ns;
    h.nn = nn;
    h.npx = s->cam.W * s->cam.H;
    h.cam = s->cam;
    h.pcg_iters = s->cfg.pcg_iters;
    h.gn_iters = s->cfg.gn_iters;
    h.debug_iter = s->cfg.debug_iter;
    h.jac_dtype = s->cfg.jac_dtype;
    h.rigid_iters = s->cfg.rigid_iters;
    h.edge_gate = s->cfg.edge_gate;
    h.dist2 = s->cfg.corr_dist * s->cfg.corr_dist;
    h.cosn = s->cfg.corr_normal;
    h.lambda = s->cfg.lambda_reg;
    h.mu = s->cfg.damping;
    h.vis_mode = s->cfg.visibility;
    h.splat = s->cfg.splat;
    h.stable_conf = s->cfg.stable_conf;
    h.recent = s->cfg.recent_frames;
    h.t_now = s->t_now;
    s->fuse_mem.release();
    s->fz4 = nullptr;
    s->fused = false;

    // nodes: positions in the caller's order on the host, the library's order
    std::vector<float> hin(3 * (size_t)nn), hcall(3 * (size_t)nn), hlib(3 * (size_t)nn);
    if (on_device) {
        SWGN_HIP(hipMemcpyAsync(hin.data(), node_pos, sizeof(float) * 3 * nn, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipStreamSynchronize(st));
    } else {
        std::memcpy(hin.data(), node_pos, sizeof(float) * 3 * nn);
    }
    if (!keep_order) s->node_perm = morton_order(hin, nn);
    const std::vector<int>& perm = s->node_perm;
    s->node_inv.assign((size_t)nn, 0);
    for (int k = 0; k < nn; ++k) s->node_inv[(size_t)perm[k]] = k;
    for (int k = 0; k < nn; ++k)
        for (int a = 0; a < 3; ++a) {
            if (keep_order) {
                hlib[3 * k + a] = hin[3 * k + a];
                hcall[3 * (size_t)perm[k] + a] = hin[3 * k + a];
            } else {
                hcall[3 * k + a] = hin[3 * k + a];
                hlib[3 * k + a] = hin[3 * (size_t)perm[k] + a];
            }
        }
    int* d_id = G.alloc<int>(nn);
    int* d_inv = G.alloc<int>(nn);
    SWGN_HIP(hipMemcpyAsync(d_id, perm.data(), sizeof(int) * nn, hipMemcpyHostToDevice, st));
    SWGN_HIP(hipMemcpyAsync(d_inv, s->node_inv.data(), sizeof(int) * nn, hipMemcpyHostToDevice, st));
    s->d_node_id = d_id;
    s->d_node_inv = d_inv;
    float* pos_in = tmp.alloc<float>(3 * (size_t)nn);
    SWGN_HIP(hipMemcpyAsync(pos_in, hlib.data(), sizeof(float) * 3 * nn, hipMemcpyHostToDevice, st));
    float4* pref = G.alloc<float4>(nn);
    launch_positions_to_f4(nn, pos_in, pref, st);
    float* pos_call = tmp.alloc<float>(3 * (size_t)nn);
    SWGN_HIP(hipMemcpyAsync(pos_call, hcall.data(), sizeof(float) * 3 * nn, hipMemcpyHostToDevice, st));
    float4* pcall = tmp.alloc<float4>(nn);
    launch_positions_to_f4(nn, pos_call, pcall, st);
    h.pref = pref;
    h.rq = G.alloc<float4>(nn);
    h.tt = G.alloc<float4>(nn);
    h.dq = G.alloc<float4>(2 * (size_t)nn);
    h.cl = G.alloc<float4>(nn);
    float* se3_in = nullptr;
    if (node_se3) {
        std::vector<float> hse((size_t)12 * nn), hsl((size_t)12 * nn);
        if (on_device) {
            SWGN_HIP(hipMemcpyAsync(hse.data(), node_se3, sizeof(float) * 12 * nn, hipMemcpyDeviceToHost, st));
            SWGN_HIP(hipStreamSynchronize(st));
        } else {
            std::memcpy(hse.data(), node_se3, sizeof(float) * 12 * nn);
        }
        for (int k = 0; k < nn; ++k)
            std::memcpy(&hsl[12 * (size_t)k], &hse[12 * (size_t)perm[k]], 12 * sizeof(float));
        se3_in = tmp.alloc<float>(12 * (size_t)nn);
        SWGN_HIP(hipMemcpyAsync(se3_in, hsl.data(), sizeof(float) * 12 * nn, hipMemcpyHostToDevice, st));
        SWGN_HIP(hipStreamSynchronize(st));                  // (the host copy goes out of scope)
    }
    if (keep_rq) {
        // the node state as it is (a rebuild after a geometry update)
        SWGN_HIP(hipMemcpyAsync(h.rq, keep_rq, sizeof(float4) * nn, hipMemcpyDeviceToDevice, st));
        SWGN_HIP(hipMemcpyAsync(h.tt, keep_tt, sizeof(float4) * nn, hipMemcpyDeviceToDevice, st));
        launch_tables_from_state(nn, pref, h.rq, h.tt, h.dq, h.cl, st);
    } else {
        launch_nodes_from_se3(nn, se3_in, pref, h.rq, h.tt, h.dq, h.cl, st);
    }

    // skinning and node graph: equal distances go to the lower caller index
    // (the skinning scans the library's order and orders candidates by
    // caller index; the graph scans the caller's order), then renumbered
    int4* idx_in = tmp.alloc<int4>(ns);
    float4* w_in = tmp.alloc<float4>(ns);
    const float sig = s->cfg.node_sigma;
    float4* boxes = tmp.alloc<float4>(knn_box_count(nn));
    launch_knn_skin(ns, s->in_pos, nn, pref, d_id, boxes, 1.0f / (2.0f * sig * sig), idx_in, w_in, st);
    launch_map_ids(reinterpret_cast<int*>(idx_in), 4 * ns, d_inv, st);
    int* nbr_call = tmp.alloc<int>(8 * (size_t)nn);
    launch_node_graph(nn, pcall, nbr_call, st);
    int* nbr = G.alloc<int>(8 * (size_t)nn);
    {
        std::vector<int> hn((size_t)8 * nn), hl((size_t)8 * nn);
        SWGN_HIP(hipMemcpyAsync(hn.data(), nbr_call, sizeof(int) * 8 * nn, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipStreamSynchronize(st));
        for (int k = 0; k < nn; ++k)
            for (int q = 0; q < 8; ++q) hl[8 * (size_t)k + q] = s->node_inv[(size_t)hn[8 * (size_t)perm[k] + q]];
        SWGN_HIP(hipMemcpyAsync(nbr, hl.data(), sizeof(int) * 8 * nn, hipMemcpyHostToDevice, st));
        SWGN_HIP(hipStreamSynchronize(st));
    }
    h.nbr = nbr;

    // order surfels by node set
    const int npad = pow2_at_least(ns, 1024);
    uint64_t* key = tmp.alloc<uint64_t>(npad);
    uint32_t* val = tmp.alloc<uint32_t>(npad);
    launch_tuple_keys(ns, npad, idx_in, key, val, st);
    sort_pairs(key, val, npad, st);
    h.pitch = (ns + 255) & ~255;
    float* spx = G.alloc<float>(h.pitch); float* spy = G.alloc<float>(h.pitch); float* spz = G.alloc<float>(h.pitch);
    float* snx = G.alloc<float>(h.pitch); float* sny = G.alloc<float>(h.pitch); float* snz = G.alloc<float>(h.pitch);
    int4* sidx = G.alloc<int4>(h.pitch);
    float4* sw = G.alloc<float4>(h.pitch);
    int* sorig = G.alloc<int>(h.pitch);
    h.px = spx; h.py = spy; h.pz = spz; h.nx = snx; h.ny = sny; h.nz = snz;
    h.idx = sidx; h.w = sw; h.orig = sorig;
    h.radius = G.alloc<float>(h.pitch);
    h.conf = G.alloc<float>(h.pitch);
    h.t_obs = G.alloc<int>(h.pitch);
    int* sinv = G.alloc<int>(std::max(1, ns));
    h.inv = sinv;
    int* flag = tmp.alloc<int>(ns + 1);
    int* fpos = tmp.alloc<int>(ns + 1);
    int* scan_tmp = tmp.alloc<int>(scan_tmp_size(std::max(10 * ns, 64 * nn) + 16));
    launch_permute_surfels(ns, 0, key, val, s->in_pos, s->in_nrm, idx_in, w_in, spx, spy, spz, snx, sny, snz,
                           sidx, sw, sorig, flag, st);
    launch_fuse_gather(ns, sorig, s->in_rad, s->in_conf, s->in_tobs, h.radius, h.conf, h.t_obs, sinv, st);
    exclusive_scan(flag, fpos, ns, scan_tmp, st);
    s->nsets = read_scalar(fpos + ns, st);
    int* set_start = tmp.alloc<int>(s->nsets + 1);      // runs of one node set
    launch_run_starts(ns, flag, fpos, set_start, st);

    // upper block pattern: every pair of a surfel's node set, every graph edge
    const int words = (nn + 31) / 32;
    uint32_t* bm = tmp.alloc<uint32_t>((size_t)nn * words);
    launch_fill_i32(reinterpret_cast<int*>(bm), nn * words, 0, st);
    launch_pattern(s->nsets, key, set_start, nn, nbr, bm, words, st);
    int* rcnt = tmp.alloc<int>(nn);
    launch_row_counts(nn, bm, words, rcnt, st);
    int* row_ptr = G.alloc<int>(nn + 1);
    exclusive_scan(rcnt, row_ptr, nn, scan_tmp, st);
    h.nb = read_scalar(row_ptr + nn, st);
    h.noff = h.nb - nn;
    int* col_idx = G.alloc<int>(h.nb);
    int* blk_row = G.alloc<int>(h.nb);
    launch_row_fill(nn, bm, words, row_ptr, col_idx, blk_row, st);
    h.row_ptr = row_ptr; h.col_idx = col_idx; h.blk_row = blk_row;
    int* offlist = G.alloc<int>(std::max(1, h.noff));
    launch_offlist(h.nb, blk_row, col_idx, offlist, st);
    h.offlist = offlist;

    build_segments(s, h, key, set_start, fpos, s->nsets, sidx, row_ptr, col_idx, G, tmp);

    // in-edges of every node (j with the node in N_j), ascending j
    const int npad_i = pow2_at_least(8 * (int64_t)nn, 1024);
    uint64_t* ikey = tmp.alloc<uint64_t>(npad_i);
    uint32_t* ival = tmp.alloc<uint32_t>(npad_i);
    int* icount = tmp.alloc<int>(nn);
    launch_fill_i32(icount, nn, 0, st);
    launch_in_edge_keys(nn, npad_i, nbr, ikey, ival, icount, st);
    sort_pairs(ikey, ival, npad_i, st);
    int* in_ptr = G.alloc<int>(nn + 1);
    exclusive_scan(icount, in_ptr, nn, scan_tmp, st);
    int* in_list = G.alloc<int>(8 * (size_t)nn);
    launch_in_edge_store(8 * nn, ival, in_list, st);
    h.in_ptr = in_ptr; h.in_list = in_list;

    // full symmetric rows for the matrix product, in ELL layout
    const int npad_t = pow2_at_least(h.nb, 1024);
    uint64_t* tkey = tmp.alloc<uint64_t>(npad_t);
    uint32_t* tval = tmp.alloc<uint32_t>(npad_t);
    int* tcount = tmp.alloc<int>(nn);
    launch_fill_i32(tcount, nn, 0, st);
    launch_transpose_keys(h.nb, npad_t, blk_row, col_idx, tkey, tval, tcount, st);
    sort_pairs(tkey, tval, npad_t, st);
    int* tstart = tmp.alloc<int>(nn + 1);
    exclusive_scan(tcount, tstart, nn, scan_tmp, st);
    int* fcount = tmp.alloc<int>(nn);
    launch_full_counts(nn, row_ptr, tcount, fcount, st);
    int* frow_ptr = tmp.alloc<int>(nn + 1);
    exclusive_scan(fcount, frow_ptr, nn, scan_tmp, st);
    const int nf = 2 * h.nb - nn;
    uint32_t* fblk = tmp.alloc<uint32_t>(nf);
    int* fcol = tmp.alloc<int>(nf);
    launch_full_rows(nn, h.noff, row_ptr, col_idx, tcount, tstart, frow_ptr, tkey, tval, fblk, fcol, st);
    {
        std::vector<int> hrow(nn + 1);
        SWGN_HIP(hipMemcpyAsync(hrow.data(), frow_ptr, sizeof(int) * (nn + 1), hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipStreamSynchronize(st));
        int wmax = 1;
        for (int k = 0; k < nn; ++k) wmax = std::max(wmax, hrow[k + 1] - hrow[k]);
        h.ell_w = (wmax + 7) & ~7;
    }
    uint32_t* ell_blk = G.alloc<uint32_t>((size_t)nn * h.ell_w);
    int* ell_col = G.alloc<int>((size_t)nn * h.ell_w);
    launch_ell(nn, h.ell_w, frow_ptr, fblk, fcol, ell_blk, ell_col, st);
    h.ell_blk = ell_blk; h.ell_col = ell_col;
    int* slot_u = G.alloc<int>(h.nb);
    int* slot_t = G.alloc<int>(h.nb);
    launch_fill_i32(slot_t, h.nb, -1, st);
    launch_ell_slots(nn, h.ell_w, ell_blk, slot_u, slot_t, st);
    h.slot_u = slot_u; h.slot_t = slot_t;

    // capture buffers, only when an iteration is to be captured
    s->dbg_index = nullptr;
    s->dbg_H = s->dbg_g = s->dbg_x = s->dbg_J = nullptr;
    if (s->cfg.debug_iter >= 0) {
        s->dbg_index = G.alloc<int>(h.npx);
        h.dbg_corr = G.alloc<int>(h.npx);
        h.dbg_live = G.alloc<float>(6 * (size_t)ns);      // live positions, then live normals
        s->dbg_H = G.alloc<float>(36 * (size_t)h.nb);
        s->dbg_g = G.alloc<float>(6 * (size_t)nn);
        s->dbg_x = G.alloc<float>(6 * (size_t)nn);
        s->dbg_J = G.alloc<float>(32 * (size_t)h.pitch);
        h.J = s->dbg_J;
    }

    // the stream's own workspace
    s->ws_bytes = carve_workspace(h, nullptr);
    char* ws = static_cast<char*>(s->ws_mem.raw(s->ws_bytes));
    carve_workspace(h, ws);

    s->h = h;
    SWGN_HIP(hipGetLastError());
    SWGN_HIP(hipStreamSynchronize(st));
    publish_desc(s);
    s->graph_set = true;
}

double model_bytes(const FrameDesc& h, int gn_iters, int64_t n_corr_total) {
    // algorithmic bytes of one frame: data each kernel must read or write at least
    const double ns = h.ns, nn = h.nn, nb = h.nb, npx = h.npx;
    double per_iter = 0.0;
    per_iter += 48.0 * ns + 8.0 * ns + 8.0 * npx;                 // warp + z-buffer (+ clear)
    per_iter += 60.0 * ns + 8.0 * ns + 16.0 * ns;                  // correspondence + J (in LDS)
    per_iter += 2.0 * 4.0 * (double)h.part_floats + 144.0 * nb + 24.0 * nn;  // segment Grams + blocks
    per_iter += 144.0 * nn + 288.0 * nn;                          // block-Jacobi
    per_iter += h.pcg_iters * (144.0 * nb + 7.0 * 24.0 * nn);     // PCG
    (void)n_corr_total;
    return gn_iters * per_iter + 20.0 * npx;
}

}  // namespace

namespace swgn {
namespace rt {

// One launch of `stage` over the streams; a stream contributes no tiles when
// it has no work in it (its Gauss-Newton or PCG iterations are done).
void run_stage(Executor& ex, int stage, const std::vector<sw_stream>& ss, const std::vector<int>& its, int pcg_it,
               const DepthIn* depth, bool timing, std::vector<int>& ev_stage, bool update) {
    Batch b{};
    b.n = (int)ss.size();
    b.pcg_it = pcg_it;
    b.update = update ? 1 : 0;
    int64_t rows = 0;
    for (int i = 0; i < b.n; ++i)
        if (its[i] >= 0) rows += ss[i]->h.nn;
    const int variant = ex.variant_of(stage, rows);
    b.order = (variant & kVarXcd) ? kOrderXcd : kOrderLinear;
    b.wide = (variant & kVarWide) ? 1 : 0;
    int off = 0;
    for (int i = 0; i < b.n; ++i) {
        const FrameDesc& h = ss[i]->h;
        b.off[i] = off;
        b.d[i] = ss[i]->d_desc;
        b.it[i] = (int8_t)its[i];
        int t = stage_tiles(stage, h, variant);
        if (its[i] < 0) t = 0;
        // products of iteration pcg_it, finish of pcg_it, fused finish of pcg_it - 1 + products
        if ((stage == kStSpmv || stage == kStUpdate) && pcg_it >= h.pcg_iters) t = 0;
        if (stage == kStPcgStep && (pcg_it < 1 || pcg_it > h.pcg_iters)) t = 0;
        // streams with PCG iterations are moved by their last finish
        if (stage == kStNodeUpdate && h.pcg_iters > 0) t = 0;
        off += t;
    }
    b.off[b.n] = off;
    if (off == 0) return;
    for (int i = 0; i < b.n; ++i) b.splat |= (its[i] >= 0 && ss[i]->h.splat) ? 1 : 0;
    if (timing) {
        SWGN_HIP(hipEventRecord(ex.event(ev_stage.size()), ex.st));
        ev_stage.push_back(stage);
    }
    switch (stage) {
        case kStDepth: case kStWarp: case kStCorr:
        case kStRigidWarp: case kStRigidSys: case kStRigidSolve: case kStRigidCompose:
            launch_frame_stage(stage, b, depth, ex.st);
            break;
        case kStAsmSeg: case kStAsmFold: launch_asm_stage(stage, b, ex.st); break;
        default: launch_solve_stage(stage, b, ex.stats_dev, ex.st); break;
    }
    if (timing) {
        SWGN_HIP(hipEventRecord(ex.event(ev_stage.size()), ex.st));
        ev_stage.push_back(-1);
    }
}

// Depth preprocessing of a frame for each stream (host images are copied into
// the streams' workspaces first).
void enqueue_depth(Executor& ex, const std::vector<sw_stream>& ss, const float* const* depths, int32_t on_device,
                   bool timing, std::vector<int>& ev) {
    DepthIn din{};
    const int n = (int)ss.size();
    for (int i = 0; i < n; ++i) {
        const FrameDesc& h = ss[i]->h;
        ++ss[i]->depth_gen;
        if (!on_device) {
            copy_in(h.depth, depths[i], sizeof(float) * h.npx, 0, ex.st);
            din.p[i] = h.depth;
        } else {
            din.p[i] = depths[i];
        }
    }
    std::vector<int> its(n, 0);
    run_stage(ex, kStDepth, ss, its, 0, &din, timing, ev);
}

// The rigid alignment of every stream whose config asks for it: rigid_iters
// steps (warp into the index map, 6x6 sums, solve), then T composed into the
// nodes. Runs after the depth preprocessing, before the first Gauss-Newton
// iteration.
void enqueue_rigid(Executor& ex, const std::vector<sw_stream>& ss, bool timing, std::vector<int>& ev) {
    const int n = (int)ss.size();
    int rmax = 0;
    for (sw_stream s : ss) rmax = std::max(rmax, s->cfg.rigid_iters);
    if (rmax == 0) return;
    std::vector<int> its(n, -1);
    for (int r = 0; r < rmax; ++r) {
        for (int i = 0; i < n; ++i) its[i] = r < ss[i]->cfg.rigid_iters ? r : -1;
        run_stage(ex, kStRigidWarp, ss, its, 0, nullptr, timing, ev);
        run_stage(ex, kStRigidSys, ss, its, 0, nullptr, timing, ev);
        run_stage(ex, kStRigidSolve, ss, its, 0, nullptr, timing, ev);
    }
    for (int i = 0; i < n; ++i) its[i] = ss[i]->cfg.rigid_iters > 0 ? 0 : -1;
    run_stage(ex, kStRigidCompose, ss, its, 0, nullptr, timing, ev);
}

// One Gauss-Newton iteration for every stream with its[i] >= 0 (its[i] = the
// stream's iteration index; -1 = no work), with the captures the streams'
// configs ask for. Sets captured[i] when stream i's capture completed.
void enqueue_iteration(Executor& ex, const std::vector<sw_stream>& ss, const std::vector<int>& its, bool timing,
                       std::vector<int>& ev, std::vector<char>& captured) {
    hipStream_t st = ex.st;
    const int n = (int)ss.size();
    int pmax = 0;
    for (int i = 0; i < n; ++i)
        if (its[i] >= 0) pmax = std::max(pmax, ss[i]->h.pcg_iters);
    auto capturing = [&](int i) { return its[i] >= 0 && its[i] == ss[i]->cfg.debug_iter; };
    run_stage(ex, kStWarp, ss, its, 0, nullptr, timing, ev);
    for (int i = 0; i < n; ++i) {
        if (!capturing(i)) continue;
        sw_stream s = ss[i];
        launch_export_index_map(s->h.npx, s->h.zbuf, s->dbg_index, st);
        launch_fill_i32(s->h.dbg_corr, s->h.npx, -1, st);
    }
    run_stage(ex, kStCorr, ss, its, 0, nullptr, timing, ev);
    run_stage(ex, kStAsmSeg, ss, its, 0, nullptr, timing, ev);
    run_stage(ex, kStAsmFold, ss, its, 0, nullptr, timing, ev);
    for (int i = 0; i < n; ++i) {
        if (!capturing(i)) continue;
        // the solve step updates the node state: keep this iteration's system first
        sw_stream s = ss[i];
        const FrameDesc& h = s->h;
        SWGN_HIP(hipMemcpyAsync(s->dbg_H, h.H, sizeof(float) * 36 * h.nb, hipMemcpyDeviceToDevice, st));
        SWGN_HIP(hipMemcpyAsync(s->dbg_g, h.g, sizeof(float) * 6 * h.nn, hipMemcpyDeviceToDevice, st));
    }
    // (the fold also starts PCG: block-Jacobi inverses, r_0, z_0, x = 0)
    int64_t rows = 0;
    for (int i = 0; i < n; ++i)
        if (its[i] >= 0) rows += ss[i]->h.nn;
    const bool fused = ex.pcg_mode == kPcgFused ||
                       (ex.pcg_mode == kPcgAuto && (ex.variant_of(kStSpmv, rows) & kVarFused) != 0);
    if (pmax > 0) run_stage(ex, kStSpmv, ss, its, 0, nullptr, timing, ev);
    for (int pit = 1; pit <= pmax; ++pit) {
        if (fused) {
            // finish of pit - 1 and, for streams with more iterations, products of pit
            run_stage(ex, kStPcgStep, ss, its, pit, nullptr, timing, ev, true);
        } else {
            run_stage(ex, kStUpdate, ss, its, pit - 1, nullptr, timing, ev, true);
            if (pit < pmax) run_stage(ex, kStSpmv, ss, its, pit, nullptr, timing, ev);
        }
    }
    run_stage(ex, kStNodeUpdate, ss, its, 0, nullptr, timing, ev);
    for (int i = 0; i < n; ++i) {
        if (!capturing(i)) continue;
        sw_stream s = ss[i];
        SWGN_HIP(hipMemcpyAsync(s->dbg_x, s->h.x, sizeof(float) * 6 * s->h.nn, hipMemcpyDeviceToDevice, st));
        captured[i] = 1;
    }
}

// Brings back the statistics of the streams' finished frames (one launch,
// one copy, one synchronisation), fills stats / status and restores the node
// state of every stream whose frame failed numerically.
void enqueue_collect(Executor& ex, const std::vector<sw_stream>& ss) {
    const int n = (int)ss.size();
    std::vector<int> its(n, 0), ev;
    run_stage(ex, kStStatsOut, ss, its, 0, nullptr, false, ev);
    SWGN_HIP(hipMemcpyAsync(ex.stats_host, ex.stats_dev, (size_t)kStatsOutBytes * n, hipMemcpyDeviceToHost, ex.st));
}

sw_status collect_frames(Executor& ex, const std::vector<sw_stream>& ss, const float* stage_us,
                         sw_frame_stats* stats, sw_status* status) {
    enqueue_collect(ex, ss);
    SWGN_HIP(hipGetLastError());
    return finish_frames(ex, ss, stage_us, stats, status);
}

sw_status finish_frames(Executor& ex, const std::vector<sw_stream>& ss, const float* stage_us,
                        sw_frame_stats* stats, sw_status* status) {
    hipStream_t st = ex.st;
    const int n = (int)ss.size();
    SWGN_HIP(hipStreamSynchronize(st));
    sw_status rc = SW_OK;
    bool restored = false;
    for (int i = 0; i < n; ++i) {
        sw_stream s = ss[i];
        const FrameDesc& h = s->h;
        const char* slot = static_cast<const char*>(ex.stats_host) + (size_t)kStatsOutBytes * i;
        const IterStats* is = reinterpret_cast<const IterStats*>(slot);
        const int* flags = reinterpret_cast<const int*>(slot + sizeof(IterStats) * kMaxIters);
        const RigidStats* rs = reinterpret_cast<const RigidStats*>(slot + sizeof(IterStats) * kMaxIters + 16);
        const int G = s->cfg.gn_iters;
        const int Rg = s->cfg.rigid_iters;
        int64_t ncorr_total = 0;
        bool bad = (flags[0] | flags[1] | flags[2] | flags[3]) != 0;
        for (int it = 0; it < G; ++it) {
            ncorr_total += is[it].n_corr;
            if (!std::isfinite(is[it].e_data) || !std::isfinite(is[it].e_reg)) bad = true;
        }
        for (int r = 0; r < Rg; ++r)
            if (!std::isfinite(rs[r].e)) bad = true;
        if (stats) {
            sw_frame_stats& o = stats[i];
            std::memset(&o, 0, sizeof(o));
            o.iters = G;
            for (int it = 0; it < G; ++it) {
                o.e_data[it] = (float)is[it].e_data;
                o.e_reg[it] = (float)is[it].e_reg;
                o.n_corr[it] = is[it].n_corr;
                o.pcg_resid[it] = (float)is[it].pcg_resid;
            }
            o.rigid_steps = Rg;
            for (int r = 0; r < Rg; ++r) {
                o.rigid_e[r] = (float)rs[r].e;
                o.rigid_n[r] = rs[r].n;
            }
            if (stage_us)
                for (int k = 0; k < 12; ++k) o.stage_us[k] = stage_us[k];
            o.alg_bytes = model_bytes(h, G, ncorr_total);
        }
        status[i] = SW_OK;
        if (bad) {
            SWGN_HIP(hipMemcpyAsync(h.rq, h.rq_bak, sizeof(float4) * h.nn, hipMemcpyDeviceToDevice, st));
            SWGN_HIP(hipMemcpyAsync(h.tt, h.tt_bak, sizeof(float4) * h.nn, hipMemcpyDeviceToDevice, st));
            launch_tables_from_state(h.nn, h.pref, h.rq, h.tt, h.dq, h.cl, st);
            s->err = "non-finite energy, node update, non-positive-definite diagonal block or rigid system;"
                     " node transforms restored";
            status[i] = SW_ENUMERIC;
            rc = SW_ENUMERIC;
            restored = true;
        }
    }
    if (restored) SWGN_HIP(hipStreamSynchronize(st));
    return rc;
}

// Solves one frame for each stream: Gauss-Newton iteration `it` of every
// stream that has one runs in the same launches. Fills stats (n entries or
// null) and status (n entries); returns SW_OK or SW_ENUMERIC.
sw_status solve_frames(Executor& ex, const std::vector<sw_stream>& ss, const float* const* depths,
                       int32_t on_device, bool timing, sw_frame_stats* stats, sw_status* status) {
    const int n = (int)ss.size();
    ex.bucket = shape_bucket(ss);
    std::vector<int> ev;
    int gmax = 0;
    bool any_capture = false;
    for (int i = 0; i < n; ++i) {
        gmax = std::max(gmax, ss[i]->cfg.gn_iters);
        any_capture |= ss[i]->cfg.debug_iter >= 0 && ss[i]->cfg.debug_iter < ss[i]->cfg.gn_iters;
    }
    enqueue_depth(ex, ss, depths, on_device, timing, ev);
    enqueue_rigid(ex, ss, timing, ev);
    std::vector<char> captured(n, 0);
    std::vector<int> its(n, 0);
    auto body = [&]() {
        for (int it = 0; it < gmax; ++it) {
            for (int i = 0; i < n; ++i) its[i] = it < ss[i]->cfg.gn_iters ? it : -1;
            enqueue_iteration(ex, ss, its, timing, ev, captured);
        }
        enqueue_collect(ex, ss);
    };
    if (ex.graphs && !timing && !any_capture) {
        // the iterations and the statistics copy of this exact batch as one
        // graph, captured on first use and replayed while the batch and its
        // streams' buffers are unchanged
        std::vector<std::pair<sw_stream, uint64_t>> key;
        for (sw_stream s : ss) key.emplace_back(s, s->generation);
        key.emplace_back(nullptr, ex.tune_epoch);
        if (!ex.graph_exec || key != ex.graph_key) {
            ex.drop_graph();
            hipGraph_t g = nullptr;
            SWGN_HIP(hipStreamBeginCapture(ex.st, hipStreamCaptureModeThreadLocal));
            try {
                body();
            } catch (...) {
                (void)hipStreamEndCapture(ex.st, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            SWGN_HIP(hipStreamEndCapture(ex.st, &g));
            hipGraphExec_t ge = nullptr;
            const hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            SWGN_HIP(e);
            ex.graph_exec = ge;
            ex.graph_key = key;
        }
        SWGN_HIP(hipGraphLaunch(ex.graph_exec, ex.st));
    } else {
        body();
    }
    SWGN_HIP(hipGetLastError());
    float stage_us[12] = {0.f};
    if (timing) {
        SWGN_HIP(hipStreamSynchronize(ex.st));
        // events come in (start of a stage, end) pairs
        for (size_t a = 0; a + 1 < ev.size(); a += 2) {
            float ms = 0.f;
            SWGN_HIP(hipEventElapsedTime(&ms, ex.events[a], ex.events[a + 1]));
            stage_us[stage_slot(ev[a])] += 1000.f * ms;
        }
    }
    const sw_status rc = finish_frames(ex, ss, timing ? stage_us : nullptr, stats, status);
    for (int i = 0; i < n; ++i)
        if (captured[i]) ss[i]->captured = true;
    return rc;
}

}  // namespace rt
}  // namespace swgn

// The upper block pattern in the caller's node order (the library keeps its
// own): row_ptr / col_idx as for the library's, and for each caller block the
// library block it comes from and whether the two orders transpose it.
struct CallerPattern {
    std::vector<int> row_ptr, col_idx, src;
    std::vector<char> transposed;
};

static CallerPattern caller_pattern(sw_stream s) {
    const int nn = s->h.nn, nb = s->h.nb;
    std::vector<int> rp(nn + 1), ci(nb);
    hipStream_t st = s->exec.st;
    SWGN_HIP(hipMemcpyAsync(rp.data(), s->h.row_ptr, sizeof(int) * (nn + 1), hipMemcpyDeviceToHost, st));
    SWGN_HIP(hipMemcpyAsync(ci.data(), s->h.col_idx, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
    SWGN_HIP(hipStreamSynchronize(st));
    const std::vector<int>& pm = s->node_perm;
    struct Ent { int a, b, src; char tr; };
    std::vector<Ent> e((size_t)nb);
    for (int k = 0; k < nn; ++k)
        for (int q = rp[k]; q < rp[k + 1]; ++q) {
            const int A = pm[k], B = pm[ci[q]];
            e[(size_t)q] = A <= B ? Ent{A, B, q, 0} : Ent{B, A, q, 1};
        }
    std::sort(e.begin(), e.end(), [](const Ent& x, const Ent& y) { return x.a < y.a || (x.a == y.a && x.b < y.b); });
    CallerPattern out;
    out.row_ptr.assign(nn + 1, 0);
    out.col_idx.resize(nb);
    out.src.resize(nb);
    out.transposed.resize(nb);
    for (int q = 0; q < nb; ++q) {
        ++out.row_ptr[e[(size_t)q].a + 1];
        out.col_idx[q] = e[(size_t)q].b;
        out.src[q] = e[(size_t)q].src;
        out.transposed[q] = e[(size_t)q].tr;
    }
    for (int k = 0; k < nn; ++k) out.row_ptr[k + 1] += out.row_ptr[k];
    return out;
}

// The allocation-free solve (sw_solve_frame_noalloc) takes a frame's workspace
// from a static array instead of the stream's own.
namespace {

// One array per GPU, held until the process ends; its size is the largest
// frame workspace this entry point accepts.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static char* g_scratch[kScratchDevices] = {};   // device address of each GPU's copy

// The device address of `scratch` on the GPU that runs hip stream st, looked
// up once per device with that device current (the host-side name is not a
// device address).
static sw_status scratch_on(hipStream_t st, std::string& err, char** out) {
    int dev = -1;
    if (hipStreamGetDevice(st, &dev) != hipSuccess || dev < 0 || dev >= kScratchDevices)
        return fail(err, SW_EHIP, "cannot tell the device of the stream");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return fail(err, SW_EHIP, "hipGetDevice failed");
        if (cur != dev && hipSetDevice(dev) != hipSuccess) return fail(err, SW_EHIP, "hipSetDevice failed");
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return fail(err, SW_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = static_cast<char*>(p);
    }
    *out = g_scratch[dev];
    return SW_OK;
}

}  // namespace

extern "C" {

void sw_config_default(sw_config* c) {
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->width = 640;
    c->height = 480;
    c->fx = 570.f; c->fy = 570.f; c->cx = 320.f; c->cy = 240.f;
    c->gn_iters = 10;
    c->pcg_iters = 10;
    c->lambda_reg = 5.0f;
    c->node_sigma = 0.025f;
    c->corr_dist = 0.05f;
    c->corr_normal = 0.5f;
    c->edge_gate = 0.03f;
    c->damping = 1e-4f;
    c->jac_dtype = 0;
    c->dot_fp64 = 1;
    c->debug_iter = -1;
    c->stage_timing = 0;
    c->rigid_iters = 0;
    c->visibility = 0;
    c->stable_conf = 10.0f;
    c->recent_frames = 2;
    c->fusion_dist = 0.001f;
    c->fusion_normal = 0.85f;
    c->warp_eps = 0.2f;
    c->append_nn = 0.3f;
    c->t_low_confid = 30;
    c->splat = 0;
}

const char* sw_status_string(sw_status st) {
    switch (st) {
        case SW_OK: return "ok";
        case SW_EINVAL: return "invalid argument";
        case SW_ESTATE: return "invalid call order";
        case SW_ENOMEM: return "out of memory";
        case SW_EHIP: return "HIP runtime error";
        case SW_ENUMERIC: return "numerical failure";
        default: return "unknown status";
    }
}

const char* sw_last_error(sw_stream s) { return s ? s->err.c_str() : "null stream"; }

sw_status sw_create_stream(const sw_config* cfg, void* hip_stream, sw_stream* out) {
    if (!out) return SW_EINVAL;
    *out = nullptr;
    std::string why;
    sw_status cs = check_config(cfg, why);
    if (cs != SW_OK) return cs;
    sw_stream_s* s = new (std::nothrow) sw_stream_s();
    if (!s) return SW_ENOMEM;
    sw_status rc = guarded(s->err, [&]() -> sw_status {
        s->cfg = *cfg;
        s->cam = Cam{cfg->width, cfg->height, cfg->fx, cfg->fy, cfg->cx, cfg->cy};
        s->exec.init(hip_stream);
        s->d_desc = s->frame_mem.alloc<FrameDesc>(1);
        void* h = nullptr;
        SWGN_HIP(hipHostMalloc(&h, sizeof(FrameDesc), hipHostMallocDefault));
        s->h_pinned = static_cast<FrameDesc*>(h);
        return SW_OK;
    });
    if (rc != SW_OK) {
        delete s;
        return rc;
    }
    *out = s;
    return SW_OK;
}

sw_status sw_destroy_stream(sw_stream s) {
    if (!s) return SW_OK;
    if (s->server) server_forget(s->server, s);
    if (s->exec.st) (void)hipStreamSynchronize(s->exec.st);
    delete s;
    return SW_OK;
}

sw_status sw_set_reference_surfels(sw_stream s, int64_t n, const float* pos, const float* nrm, int32_t on_device) {
    if (!s) return SW_EINVAL;
    if (s->server) return fail(s->err, SW_ESTATE, "the stream is attached to a server");
    if (n < 1 || n >= kMaxSurfels) return fail(s->err, SW_EINVAL, "surfel count out of range");
    if (!pos || !nrm) return fail(s->err, SW_EINVAL, "surfel pointers must not be NULL");
    if (on_device != 0 && on_device != 1) return fail(s->err, SW_EINVAL, "on_device must be 0 or 1");
    return guarded(s->err, [&]() -> sw_status {
        s->graph_mem.release();
        s->ws_mem.release();
        s->graph_set = false;
        s->captured = false;
        ++s->generation;
        s->surf_mem.release();
        s->surfels_set = false;
        s->ns = n;
        s->fuse_mem.release();
        s->fz4 = nullptr;
        s->fused = false;
        s->in_pos = s->surf_mem.alloc<float>(3 * (size_t)n);
        s->in_nrm = s->surf_mem.alloc<float>(3 * (size_t)n);
        copy_in(s->in_pos, pos, sizeof(float) * 3 * n, on_device, s->exec.st);
        copy_in(s->in_nrm, nrm, sizeof(float) * 3 * n, on_device, s->exec.st);
        // attributes: radius 0, confidence 1, last observed and initialisation frame 0
        s->in_rad = s->surf_mem.alloc<float>(n);
        s->in_conf = s->surf_mem.alloc<float>(n);
        s->in_tobs = s->surf_mem.alloc<int>(n);
        s->in_tinit = s->surf_mem.alloc<int>(n);
        launch_fill_i32(reinterpret_cast<int*>(s->in_rad), (int)n, 0, s->exec.st);
        launch_fill_i32(reinterpret_cast<int*>(s->in_conf), (int)n, 0x3f800000, s->exec.st);
        launch_fill_i32(s->in_tobs, (int)n, 0, s->exec.st);
        launch_fill_i32(s->in_tinit, (int)n, 0, s->exec.st);
        SWGN_HIP(hipStreamSynchronize(s->exec.st));
        s->surfels_set = true;
        return SW_OK;
    });
}

sw_status sw_set_node_graph(sw_stream s, int32_t n_nodes, const float* node_pos, const float* node_se3,
                            int32_t on_device) {
    if (!s) return SW_EINVAL;
    if (s->server) return fail(s->err, SW_ESTATE, "the stream is attached to a server");
    if (!s->surfels_set) return fail(s->err, SW_ESTATE, "reference surfels must be set before the node graph");
    if (n_nodes < 9 || n_nodes > kMaxNodes) return fail(s->err, SW_EINVAL, "n_nodes must be in [9, 32768]");
    if (!node_pos) return fail(s->err, SW_EINVAL, "node positions must not be NULL");
    if (on_device != 0 && on_device != 1) return fail(s->err, SW_EINVAL, "on_device must be 0 or 1");
    return guarded(s->err, [&]() -> sw_status {
        build_graph(s, n_nodes, node_pos, node_se3, on_device, nullptr, nullptr, false);
        return SW_OK;
    });
}

sw_status sw_set_node_se3(sw_stream s, const float* node_se3, int32_t n, int32_t on_device) {
    if (!s) return SW_EINVAL;
    if (s->server) return fail(s->err, SW_ESTATE, "the stream is attached to a server");
    if (!s->graph_set) return fail(s->err, SW_ESTATE, "node graph not set");
    if (n != s->h.nn || !node_se3) return fail(s->err, SW_EINVAL, "need n_nodes transforms");
    if (on_device != 0 && on_device != 1) return fail(s->err, SW_EINVAL, "on_device must be 0 or 1");
    return guarded(s->err, [&]() -> sw_status {
        Arena tmp;
        float* d = tmp.alloc<float>(12 * (size_t)n);
        const FrameDesc& h = s->h;
        std::vector<float> in((size_t)12 * n), lib((size_t)12 * n);
        if (on_device) {
            SWGN_HIP(hipMemcpyAsync(in.data(), node_se3, sizeof(float) * 12 * n, hipMemcpyDeviceToHost, s->exec.st));
            SWGN_HIP(hipStreamSynchronize(s->exec.st));
        } else {
            std::memcpy(in.data(), node_se3, sizeof(float) * 12 * n);
        }
        for (int k = 0; k < n; ++k)             // into the library's node order
            std::memcpy(&lib[12 * (size_t)k], &in[12 * (size_t)s->node_perm[k]], 12 * sizeof(float));
        SWGN_HIP(hipMemcpyAsync(d, lib.data(), sizeof(float) * 12 * n, hipMemcpyHostToDevice, s->exec.st));
        launch_nodes_from_se3(n, d, h.pref, h.rq, h.tt, h.dq, h.cl, s->exec.st);
        SWGN_HIP(hipGetLastError());
        SWGN_HIP(hipStreamSynchronize(s->exec.st));
        return SW_OK;
    });
}

sw_status sw_solve_frame(sw_stream s, const float* depth, int32_t on_device, sw_frame_stats* stats) {
    if (!s) return SW_EINVAL;
    if (s->server) return fail(s->err, SW_ESTATE, "the stream is attached to a server");
    if (!s->graph_set) return fail(s->err, SW_ESTATE, "surfels and node graph must be set before solving");
    if (!depth) return fail(s->err, SW_EINVAL, "depth must not be NULL");
    if (on_device != 0 && on_device != 1) return fail(s->err, SW_EINVAL, "on_device must be 0 or 1");
    return guarded(s->err, [&]() -> sw_status {
        std::vector<sw_stream> one{s};
        sw_status st1 = SW_OK;
        return solve_frames(s->exec, one, &depth, on_device, s->cfg.stage_timing != 0, stats, &st1);
    });
}

// ---- the solve without allocation (the scratch array is defined above) ----

sw_status sw_solve_frame_noalloc(sw_stream s, const float* depth, int32_t on_device, sw_frame_stats* stats) {
    if (!s) return SW_EINVAL;
    if (s->server) return fail(s->err, SW_ESTATE, "the stream is attached to a server");
    if (!s->graph_set) return fail(s->err, SW_ESTATE, "surfels and node graph must be set before solving");
    if (!depth) return fail(s->err, SW_EINVAL, "depth must not be NULL");
    if (on_device != 0 && on_device != 1) return fail(s->err, SW_EINVAL, "on_device must be 0 or 1");
    if (s->ws_bytes > kScratchBytes)
        return fail(s->err, SW_EINVAL, "the frame workspace (" + std::to_string(s->ws_bytes) +
                                           " bytes) exceeds the static scratch (" + std::to_string(kScratchBytes) +
                                           " bytes)");
    char* base = nullptr;
    if (scratch_on(s->exec.st, s->err, &base) != SW_OK) return SW_EHIP;
    return guarded(s->err, [&]() -> sw_status {
        // the frame's workspace carved from the scratch for this call; the
        // stream's descriptor points back at its own workspace afterwards
        const FrameDesc own = s->h;
        carve_workspace(s->h, base);
        publish_desc(s);
        sw_status r = SW_OK;
        try {
            std::vector<sw_stream> one{s};
            sw_status st1 = SW_OK;
            r = solve_frames(s->exec, one, &depth, on_device, s->cfg.stage_timing != 0, stats, &st1);
        } catch (...) {
            (void)hipStreamSynchronize(s->exec.st);
            s->h = own;
            publish_desc(s);
            throw;
        }
        SWGN_HIP(hipStreamSynchronize(s->exec.st));
        s->h = own;
        publish_desc(s);
        return r;
    });
}

sw_status sw_get_node_se3(sw_stream s, float* out, int32_t capacity) {
    if (!s) return SW_EINVAL;
    if (s->server) server_quiesce(s->server, s);
    if (!s->graph_set) return fail(s->err, SW_ESTATE, "node graph not set");
    if (!out || capacity < s->h.nn) return fail(s->err, SW_EINVAL, "output capacity below n_nodes");
    return guarded(s->err, [&]() -> sw_status {
        Arena tmp;
        const int nn = s->h.nn;
        float* d = tmp.alloc<float>(12 * (size_t)nn);
        launch_node_se3_out(nn, s->h.rq, s->h.tt, d, s->exec.st);
        std::vector<float> lib((size_t)12 * nn);
        SWGN_HIP(hipMemcpyAsync(lib.data(), d, sizeof(float) * 12 * nn, hipMemcpyDeviceToHost, s->exec.st));
        SWGN_HIP(hipStreamSynchronize(s->exec.st));
        for (int k = 0; k < nn; ++k)            // back to the caller's node order
            std::memcpy(out + 12 * (size_t)s->node_perm[k], &lib[12 * (size_t)k], 12 * sizeof(float));
        return SW_OK;
    });
}

// ---- surfel attributes and depth-map fusion ----

sw_status sw_set_surfel_attributes(sw_stream s, int64_t n, const float* radius, const float* confidence,
                                   const int32_t* t_observed, const int32_t* t_init, int32_t on_device) {
    if (!s) return SW_EINVAL;
    if (s->server) return fail(s->err, SW_ESTATE, "the stream is attached to a server");
    if (!s->surfels_set) return fail(s->err, SW_ESTATE, "surfels must be set first");
    if (n != s->ns) return fail(s->err, SW_EINVAL, "n must equal the surfel count");
    if (on_device != 0 && on_device != 1) return fail(s->err, SW_EINVAL, "on_device must be 0 or 1");
    return guarded(s->err, [&]() -> sw_status {
        hipStream_t st = s->exec.st;
        if (radius) {
            // a disc needs a radius >= 0 (0 = an unsized point); anything else
            // is refused before any attribute changes
            std::vector<float> hr((size_t)n);
            if (on_device) {
                SWGN_HIP(hipMemcpyAsync(hr.data(), radius, sizeof(float) * n, hipMemcpyDeviceToHost, st));
                SWGN_HIP(hipStreamSynchronize(st));
            } else {
                std::memcpy(hr.data(), radius, sizeof(float) * n);
            }
            for (int64_t i = 0; i < n; ++i)
                if (!(hr[i] >= 0.f) || !std::isfinite(hr[i]))
                    return fail(s->err, SW_EINVAL, "radius " + std::to_string(i) + " is negative or not finite");
        }
        if (radius) copy_in(s->in_rad, radius, sizeof(float) * n, on_device, st);
        if (confidence) copy_in(s->in_conf, confidence, sizeof(float) * n, on_device, st);
        if (t_observed) copy_in(s->in_tobs, t_observed, sizeof(int32_t) * n, on_device, st);
        if (t_init) copy_in(s->in_tinit, t_init, sizeof(int32_t) * n, on_device, st);
        if (s->graph_set)
            launch_fuse_gather((int)s->ns, s->h.orig, s->in_rad, s->in_conf, s->in_tobs, s->h.radius, s->h.conf,
                               s->h.t_obs, const_cast<int*>(s->h.inv), st);
        SWGN_HIP(hipGetLastError());
        SWGN_HIP(hipStreamSynchronize(st));
        return SW_OK;
    });
}

sw_status sw_get_surfel_attributes(sw_stream s, float* radius, float* confidence, int32_t* t_observed,
                                   int32_t* t_init) {
    if (!s) return SW_EINVAL;
    if (s->server) server_quiesce(s->server, s);
    if (!s->surfels_set) return fail(s->err, SW_ESTATE, "surfels not set");
    return guarded(s->err, [&]() -> sw_status {
        hipStream_t st = s->exec.st;
        const size_t n = (size_t)s->ns;
        if (radius) SWGN_HIP(hipMemcpyAsync(radius, s->in_rad, sizeof(float) * n, hipMemcpyDeviceToHost, st));
        if (confidence) SWGN_HIP(hipMemcpyAsync(confidence, s->in_conf, sizeof(float) * n, hipMemcpyDeviceToHost, st));
        if (t_observed) SWGN_HIP(hipMemcpyAsync(t_observed, s->in_tobs, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
        if (t_init) SWGN_HIP(hipMemcpyAsync(t_init, s->in_tinit, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipStreamSynchronize(st));
        return SW_OK;
    });
}

sw_status sw_get_reference_surfels(sw_stream s, float* pos, float* nrm) {
    if (!s) return SW_EINVAL;
    if (s->server) server_quiesce(s->server, s);
    if (!s->surfels_set) return fail(s->err, SW_ESTATE, "surfels not set");
    return guarded(s->err, [&]() -> sw_status {
        hipStream_t st = s->exec.st;
        const size_t n = (size_t)s->ns;
        if (pos) SWGN_HIP(hipMemcpyAsync(pos, s->in_pos, sizeof(float) * 3 * n, hipMemcpyDeviceToHost, st));
        if (nrm) SWGN_HIP(hipMemcpyAsync(nrm, s->in_nrm, sizeof(float) * 3 * n, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipStreamSynchronize(st));
        return SW_OK;
    });
}

sw_status sw_set_frame_time(sw_stream s, int32_t t_now) {
    if (!s) return SW_EINVAL;
    if (s->server) return fail(s->err, SW_ESTATE, "the stream is attached to a server");
    return guarded(s->err, [&]() -> sw_status {
        s->t_now = t_now;
        if (s->graph_set) {
            s->h.t_now = t_now;
            publish_desc(s);
        }
        return SW_OK;
    });
}

sw_status sw_fuse_frame(sw_stream s, const float* depth, int32_t on_device, int32_t t_now, sw_fusion_stats* stats) {
    if (!s) return SW_EINVAL;
    if (s->server) return fail(s->err, SW_ESTATE, "the stream is attached to a server");
    if (!s->graph_set) return fail(s->err, SW_ESTATE, "surfels and node graph must be set before fusing");
    if (!depth) return fail(s->err, SW_EINVAL, "depth must not be NULL");
    if (on_device != 0 && on_device != 1) return fail(s->err, SW_EINVAL, "on_device must be 0 or 1");
    return guarded(s->err, [&]() -> sw_status {
        hipStream_t st = s->exec.st;
        FrameDesc& h = s->h;
        if (!s->fz4) {
            s->fuse_mem.release();
            s->fz4 = s->fuse_mem.alloc<unsigned long long>((size_t)16 * h.npx);
            s->flive = s->fuse_mem.alloc<float>(6 * (size_t)h.pitch);
            s->fmatch = s->fuse_mem.alloc<int>(h.npx);
            s->fcount = s->fuse_mem.alloc<int>(2);
            if (!s->fcount_host) SWGN_HIP(hipHostMalloc(reinterpret_cast<void**>(&s->fcount_host), 8 * sizeof(int)));
        }
        s->t_now = t_now;
        h.t_now = t_now;
        publish_desc(s);
        // the frame's normal map (the same preprocessing as a solve)
        std::vector<sw_stream> one{s};
        std::vector<int> ev;
        enqueue_depth(s->exec, one, &depth, on_device, false, ev);
        s->fuse_gen = s->depth_gen;
        launch_fill_i32(s->fcount, 2, 0, st);
        FuseArgs a{};
        a.ns = (int)s->ns;
        a.t_now = t_now;
        a.cam = h.cam;
        const float dd = s->cfg.fusion_dist;
        a.dist2 = dd * dd;
        a.cosn = s->cfg.fusion_normal;
        a.cos_max = 0.258819045f;              // cos 75 deg
        a.idx = h.idx; a.w = h.w; a.dq = h.dq; a.orig = h.orig; a.inv = h.inv;
        a.px = const_cast<float*>(h.px); a.py = const_cast<float*>(h.py); a.pz = const_cast<float*>(h.pz);
        a.nx = const_cast<float*>(h.nx); a.ny = const_cast<float*>(h.ny); a.nz = const_cast<float*>(h.nz);
        a.radius = h.radius; a.conf = h.conf; a.t_obs = h.t_obs;
        a.nmap = h.nmap;
        a.zmap4 = s->fz4;
        const size_t P = (size_t)h.pitch;
        a.lx = s->flive; a.ly = s->flive + P; a.lz = s->flive + 2 * P;
        a.lnx = s->flive + 3 * P; a.lny = s->flive + 4 * P; a.lnz = s->flive + 5 * P;
        a.match = s->fmatch;
        a.counts = s->fcount;
        a.cpos = s->in_pos; a.cnrm = s->in_nrm; a.crad = s->in_rad; a.cconf = s->in_conf; a.ctobs = s->in_tobs;
        launch_fuse(a, st);
        SWGN_HIP(hipGetLastError());
        SWGN_HIP(hipMemcpyAsync(s->fcount_host, s->fcount, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipStreamSynchronize(st));
        s->fused = true;
        if (stats) {
            stats->n_fused = s->fcount_host[0];
            stats->n_candidates = s->fcount_host[1];
        }
        return SW_OK;
    });
}

sw_status sw_get_last_fusion(sw_stream s, int32_t* match_map, float* live_pos, float* live_nrm) {
    if (!s) return SW_EINVAL;
    if (s->server) server_quiesce(s->server, s);
    if (!s->fused || !s->graph_set) return fail(s->err, SW_ESTATE, "no fusion has run on this node graph");
    return guarded(s->err, [&]() -> sw_status {
        hipStream_t st = s->exec.st;
        const FrameDesc& h = s->h;
        if (match_map)
            SWGN_HIP(hipMemcpyAsync(match_map, s->fmatch, sizeof(int) * h.npx, hipMemcpyDeviceToHost, st));
        if (live_pos || live_nrm) {
            const size_t P = (size_t)h.pitch, n = (size_t)h.ns;
            std::vector<float> lv(6 * P);
            std::vector<int> org(n);
            SWGN_HIP(hipMemcpyAsync(lv.data(), s->flive, sizeof(float) * 6 * P, hipMemcpyDeviceToHost, st));
            SWGN_HIP(hipMemcpyAsync(org.data(), h.orig, sizeof(int) * n, hipMemcpyDeviceToHost, st));
            SWGN_HIP(hipStreamSynchronize(st));
            for (size_t i = 0; i < n; ++i)
                for (int c = 0; c < 3; ++c) {
                    if (live_pos) live_pos[3 * (size_t)org[i] + c] = lv[c * P + i];
                    if (live_nrm) live_nrm[3 * (size_t)org[i] + c] = lv[(3 + c) * P + i];
                }
        }
        SWGN_HIP(hipStreamSynchronize(st));
        return SW_OK;
    });
}

namespace {

// The append selection of the last fusion into out_* (device arrays of
// capacity max_out), or into the stream's staging arrays (capacity npx) when
// pixel is NULL; counts into stats. The caller has checked the state.
void run_append(sw_stream s, int32_t max_out, int32_t* pixel, float* pos, float* nrm, float* radius,
                float* confidence, sw_append_stats* stats) {
    hipStream_t st = s->exec.st;
    const FrameDesc& h = s->h;
    const int npx = h.npx;
    if (!s->aflag) {
        s->aflag = s->append_mem.alloc<int>(npx + 1);
        s->apos = s->append_mem.alloc<int>(npx + 1);
        s->ascan = s->append_mem.alloc<int>(scan_tmp_size(npx + 1));
        s->acount = s->append_mem.alloc<int>(4);
        s->asv = s->append_mem.alloc<float4>(npx);
        s->asn = s->append_mem.alloc<float4>(npx);
        s->apix = s->append_mem.alloc<int>(npx);
        s->apos3 = s->append_mem.alloc<float>(3 * (size_t)npx);
        s->anrm3 = s->append_mem.alloc<float>(3 * (size_t)npx);
        s->arad = s->append_mem.alloc<float>(npx);
        s->aconf = s->append_mem.alloc<float>(npx);
    }
    AppendArgs a{};
    a.cam = h.cam;
    a.nn = h.nn;
    a.eps = s->cfg.warp_eps;
    a.delta_nn = s->cfg.append_nn;
    a.inv2s2 = 1.0f / (2.0f * s->cfg.node_sigma * s->cfg.node_sigma);
    a.cos_max = 0.258819045f;              // cos 75 deg
    a.nmap = h.nmap;
    a.match = s->fmatch;
    a.cl = h.cl;
    a.pref = h.pref;
    a.node_id = s->d_node_id;
    a.node_inv = s->d_node_inv;
    a.dq = h.dq;
    a.flag = s->aflag;
    a.sv = s->asv;
    a.sn = s->asn;
    a.counts = s->acount;
    if (pixel) {
        a.max_out = max_out;
        a.out_pixel = pixel; a.out_pos = pos; a.out_nrm = nrm; a.out_rad = radius; a.out_conf = confidence;
    } else {
        a.max_out = std::min(max_out, npx);
        a.out_pixel = s->apix; a.out_pos = s->apos3; a.out_nrm = s->anrm3; a.out_rad = s->arad;
        a.out_conf = s->aconf;
    }
    launch_fill_i32(s->acount, 4, 0, st);
    launch_fill_i32(s->aflag + npx, 1, 0, st);
    launch_append(a, s->apos, s->ascan, st);
    SWGN_HIP(hipGetLastError());
    int* hc = s->fcount_host;
    SWGN_HIP(hipMemcpyAsync(hc + 2, s->acount, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
    SWGN_HIP(hipMemcpyAsync(hc + 5, s->apos + npx, sizeof(int), hipMemcpyDeviceToHost, st));
    SWGN_HIP(hipStreamSynchronize(st));
    stats->n_candidates = hc[2];
    stats->n_far = hc[3];
    stats->n_compressive = hc[4];
    stats->n_appended = hc[5];
    stats->n_written = std::min(hc[5], a.max_out);
}

sw_status append_state(sw_stream s) {
    if (s->server) return fail(s->err, SW_ESTATE, "the stream is attached to a server");
    if (!s->graph_set || !s->fused || s->fuse_gen != s->depth_gen)
        return fail(s->err, SW_ESTATE, "append candidates need a fusion as the stream's last depth frame");
    return SW_OK;
}

}  // namespace

sw_status sw_append_candidates(sw_stream s, int32_t max_out, int32_t on_device, int32_t* pixel, float* pos,
                               float* nrm, float* radius, float* confidence, sw_append_stats* stats) {
    if (!s) return SW_EINVAL;
    if (append_state(s) != SW_OK) return SW_ESTATE;
    if (max_out < 0) return fail(s->err, SW_EINVAL, "max_out must be >= 0");
    if (max_out > 0 && !(pixel && pos && nrm && radius && confidence))
        return fail(s->err, SW_EINVAL, "output pointers must not be NULL when max_out > 0");
    if (on_device != 0 && on_device != 1) return fail(s->err, SW_EINVAL, "on_device must be 0 or 1");
    return guarded(s->err, [&]() -> sw_status {
        hipStream_t st = s->exec.st;
        sw_append_stats as{};
        if (on_device && max_out > 0)
            run_append(s, max_out, pixel, pos, nrm, radius, confidence, &as);
        else
            run_append(s, on_device ? 0 : max_out, nullptr, nullptr, nullptr, nullptr, nullptr, &as);
        const int nw = as.n_written;
        if (!on_device && nw > 0) {
            SWGN_HIP(hipMemcpyAsync(pixel, s->apix, sizeof(int) * nw, hipMemcpyDeviceToHost, st));
            SWGN_HIP(hipMemcpyAsync(pos, s->apos3, sizeof(float) * 3 * nw, hipMemcpyDeviceToHost, st));
            SWGN_HIP(hipMemcpyAsync(nrm, s->anrm3, sizeof(float) * 3 * nw, hipMemcpyDeviceToHost, st));
            SWGN_HIP(hipMemcpyAsync(radius, s->arad, sizeof(float) * nw, hipMemcpyDeviceToHost, st));
            SWGN_HIP(hipMemcpyAsync(confidence, s->aconf, sizeof(float) * nw, hipMemcpyDeviceToHost, st));
            SWGN_HIP(hipStreamSynchronize(st));
        }
        if (stats) *stats = as;
        return SW_OK;
    });
}

sw_status sw_update_geometry(sw_stream s, sw_geometry_stats* stats) {
    if (!s) return SW_EINVAL;
    if (append_state(s) != SW_OK) return SW_ESTATE;
    return guarded(s->err, [&]() -> sw_status {
        hipStream_t st = s->exec.st;
        const int ns = (int)s->ns;
        const int nn = s->h.nn;
        sw_append_stats as{};
        run_append(s, s->h.npx, nullptr, nullptr, nullptr, nullptr, nullptr, &as);
        const int napp = as.n_written;
        // which existing surfels stay (caller order), and where
        Arena tmp;
        int* flag = tmp.alloc<int>(ns + 1);
        int* pos = tmp.alloc<int>(ns + 1);
        int* scan = tmp.alloc<int>(scan_tmp_size(ns + 1));
        launch_keep_mark(ns, s->in_conf, s->in_tinit, s->t_now, s->cfg.stable_conf, s->cfg.t_low_confid, flag, st);
        launch_fill_i32(flag + ns, 1, 0, st);
        exclusive_scan(flag, pos, ns + 1, scan, st);
        const int nkeep = read_scalar(pos + ns, st);
        const int64_t nnew = (int64_t)nkeep + napp;
        if (nnew < 1 || nnew >= kMaxSurfels)
            return fail(s->err, SW_EINVAL, "the update would leave no surfel or exceed the surfel limit");
        // the node state and positions, kept across the rebuild
        float4* rq = tmp.alloc<float4>(nn);
        float4* tt = tmp.alloc<float4>(nn);
        float* np3 = tmp.alloc<float>(3 * (size_t)nn);
        SWGN_HIP(hipMemcpyAsync(rq, s->h.rq, sizeof(float4) * nn, hipMemcpyDeviceToDevice, st));
        SWGN_HIP(hipMemcpyAsync(tt, s->h.tt, sizeof(float4) * nn, hipMemcpyDeviceToDevice, st));
        launch_f4_to_positions(nn, s->h.pref, np3, st);
        // the compacted caller-order arrays
        Arena fresh;
        CompactArgs c{};
        c.ns = ns; c.nkeep = nkeep; c.napp = napp; c.t_now = s->t_now;
        c.flag = flag; c.pos = pos;
        c.spos = s->in_pos; c.snrm = s->in_nrm; c.srad = s->in_rad; c.sconf = s->in_conf;
        c.stobs = s->in_tobs; c.stinit = s->in_tinit;
        c.apos = s->apos3; c.anrm = s->anrm3; c.arad = s->arad; c.aconf = s->aconf;
        c.dpos = fresh.alloc<float>(3 * (size_t)nnew);
        c.dnrm = fresh.alloc<float>(3 * (size_t)nnew);
        c.drad = fresh.alloc<float>(nnew);
        c.dconf = fresh.alloc<float>(nnew);
        c.dtobs = fresh.alloc<int>(nnew);
        c.dtinit = fresh.alloc<int>(nnew);
        launch_compact_surfels(c, st);
        SWGN_HIP(hipGetLastError());
        SWGN_HIP(hipStreamSynchronize(st));
        // swap in the new surfels (the old arrays go with `fresh`) and rebuild
        s->surf_mem.swap(fresh);
        s->ns = nnew;
        s->in_pos = c.dpos; s->in_nrm = c.dnrm; s->in_rad = c.drad; s->in_conf = c.dconf;
        s->in_tobs = c.dtobs; s->in_tinit = c.dtinit;
        build_graph(s, nn, np3, nullptr, 1, rq, tt, true);
        SWGN_HIP(hipStreamSynchronize(st));
        if (stats) {
            stats->n_removed = ns - nkeep;
            stats->n_surfels = (int32_t)nnew;
            stats->append = as;
        }
        return SW_OK;
    });
}

sw_status sw_get_live_nodes(sw_stream s, float* pos) {
    if (!s) return SW_EINVAL;
    if (s->server) server_quiesce(s->server, s);
    if (!s->graph_set) return fail(s->err, SW_ESTATE, "no node graph set");
    if (!pos) return fail(s->err, SW_EINVAL, "pos must not be NULL");
    return guarded(s->err, [&]() -> sw_status {
        hipStream_t st = s->exec.st;
        const int nn = s->h.nn;
        std::vector<float4> c(nn);
        SWGN_HIP(hipMemcpyAsync(c.data(), s->h.cl, sizeof(float4) * nn, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipStreamSynchronize(st));
        for (int k = 0; k < nn; ++k) {
            const size_t o = (size_t)s->node_perm[k];
            pos[3 * o + 0] = c[k].x;
            pos[3 * o + 1] = c[k].y;
            pos[3 * o + 2] = c[k].z;
        }
        return SW_OK;
    });
}

sw_status sw_get_sizes(sw_stream s, int64_t* n_surfels, int32_t* n_nodes, int32_t* n_blocks) {
    if (!s) return SW_EINVAL;
    if (n_surfels) *n_surfels = s->ns;
    if (n_nodes) *n_nodes = s->graph_set ? s->h.nn : 0;
    if (n_blocks) *n_blocks = s->graph_set ? s->h.nb : 0;
    return SW_OK;
}

sw_status sw_get_layout(sw_stream s, sw_layout* out) {
    if (!s || !out) return SW_EINVAL;
    if (!s->graph_set) return fail(s->err, SW_ESTATE, "node graph not set");
    std::memset(out, 0, sizeof(*out));
    out->node_sets = s->nsets;
    out->segments = s->h.nseg;
    out->packs = s->h.npack;
    out->ell_width = s->h.ell_w;
    out->fold_entries = s->nent;
    out->gram_floats = s->h.part_floats;
    return SW_OK;
}

sw_status sw_check_layout(sw_stream s, int64_t* differ) {
    if (!s) return SW_EINVAL;
    if (!s->graph_set) return fail(s->err, SW_ESTATE, "node graph not set");
    if (!differ) return fail(s->err, SW_EINVAL, "NULL output");
    return guarded(s->err, [&]() -> sw_status {
        const FrameDesc& h = s->h;
        const int ns = h.ns, nn = h.nn, nb = h.nb;
        hipStream_t st = s->exec.st;
        std::vector<int4> idx(ns);
        std::vector<int> rp(nn + 1), ci(nb);
        SWGN_HIP(hipMemcpyAsync(idx.data(), h.idx, sizeof(int4) * ns, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipMemcpyAsync(rp.data(), h.row_ptr, sizeof(int) * (nn + 1), hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipMemcpyAsync(ci.data(), h.col_idx, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipStreamSynchronize(st));
        // the sequential walk over the surfels as sorted on the device
        std::vector<uint64_t> key(ns);
        std::vector<int32_t> idx4(4 * (size_t)ns);
        for (int i = 0; i < ns; ++i) {
            int t[4] = {idx[i].x, idx[i].y, idx[i].z, idx[i].w};
            for (int k = 0; k < 4; ++k) idx4[4 * (size_t)i + k] = t[k];
            std::sort(t, t + 4);
            key[i] = ((uint64_t)t[0] << 48) | ((uint64_t)t[1] << 32) | ((uint64_t)t[2] << 16) | (uint64_t)t[3];
        }
        SegmentLayout L;
        std::string why;
        if (!segment_layout(ns, nn, nb, key.data(), idx4.data(), rp.data(), ci.data(), kCorrPack, L, why))
            return fail(s->err, SW_EINVAL, "host segment walk: " + why);
        const int nseg = h.nseg, npack = h.npack;
        const int64_t ne = s->nent;
        std::vector<int> seg(nseg + 1), ep(nb + 1), ps(npack + 1), pg(npack + 1);
        std::vector<uint16_t> mask(nseg), pos4(ns);
        std::vector<uint32_t> off(nseg + 1), es(ne), eg(ne);
        SWGN_HIP(hipMemcpyAsync(seg.data(), h.seg_start, sizeof(int) * (nseg + 1), hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipMemcpyAsync(mask.data(), h.seg_mask, sizeof(uint16_t) * nseg, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipMemcpyAsync(off.data(), h.seg_off, sizeof(uint32_t) * (nseg + 1), hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipMemcpyAsync(ep.data(), h.ent_ptr, sizeof(int) * (nb + 1), hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipMemcpyAsync(es.data(), h.ent_sub, sizeof(uint32_t) * ne, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipMemcpyAsync(eg.data(), h.ent_grad, sizeof(uint32_t) * ne, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipMemcpyAsync(ps.data(), h.pack_start, sizeof(int) * (npack + 1), hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipMemcpyAsync(pg.data(), h.pack_seg, sizeof(int) * (npack + 1), hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipMemcpyAsync(pos4.data(), h.pos4, sizeof(uint16_t) * ns, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipStreamSynchronize(st));
        auto cmp = [](const auto& a, const auto& b) -> int64_t {
            const size_t n = std::min(a.size(), b.size());
            int64_t d = (int64_t)std::max(a.size(), b.size()) - (int64_t)n;
            for (size_t i = 0; i < n; ++i) d += (int64_t)(a[i] != b[i]);
            return d;
        };
        differ[0] = cmp(seg, L.seg_start);
        differ[1] = cmp(mask, L.mask);
        differ[2] = cmp(off, L.off) + (int64_t)((uint64_t)h.part_floats != L.total);
        differ[3] = cmp(ep, L.ent_ptr);
        differ[4] = cmp(es, L.ent_sub);
        differ[5] = cmp(eg, L.ent_grad);
        differ[6] = cmp(ps, L.pack_start);
        differ[7] = cmp(pg, L.pack_seg);
        differ[8] = cmp(pos4, L.pos4);
        return SW_OK;
    });
}

sw_status sw_get_footprint(sw_stream s, int64_t* resident_bytes, int64_t* workspace_bytes) {
    if (!s) return SW_EINVAL;
    if (!s->graph_set) return fail(s->err, SW_ESTATE, "node graph not set");
    if (resident_bytes)
        *resident_bytes = (int64_t)(s->surf_mem.bytes() + s->graph_mem.bytes() + s->frame_mem.bytes() +
                                     s->setup_mem.bytes());
    if (workspace_bytes) *workspace_bytes = (int64_t)s->ws_bytes;
    return SW_OK;
}

sw_status sw_get_skinning(sw_stream s, int32_t* idx4, float* w4) {
    if (!s) return SW_EINVAL;
    if (!s->graph_set) return fail(s->err, SW_ESTATE, "node graph not set");
    return guarded(s->err, [&]() -> sw_status {
        const size_t ns = (size_t)s->ns;
        hipStream_t st = s->exec.st;
        std::vector<int4> idx(ns);
        std::vector<float4> w(ns);
        std::vector<int> orig(ns);
        SWGN_HIP(hipMemcpyAsync(idx.data(), s->h.idx, sizeof(int4) * ns, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipMemcpyAsync(w.data(), s->h.w, sizeof(float4) * ns, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipMemcpyAsync(orig.data(), s->h.orig, sizeof(int) * ns, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipStreamSynchronize(st));
        for (size_t i = 0; i < ns; ++i) {
            const size_t o = (size_t)orig[i];
            if (idx4) {
                const std::vector<int>& pm = s->node_perm;
                idx4[4 * o] = pm[idx[i].x]; idx4[4 * o + 1] = pm[idx[i].y];
                idx4[4 * o + 2] = pm[idx[i].z]; idx4[4 * o + 3] = pm[idx[i].w];
            }
            if (w4) { w4[4 * o] = w[i].x; w4[4 * o + 1] = w[i].y; w4[4 * o + 2] = w[i].z; w4[4 * o + 3] = w[i].w; }
        }
        return SW_OK;
    });
}

sw_status sw_get_node_graph(sw_stream s, int32_t* nbr8) {
    if (!s) return SW_EINVAL;
    if (!s->graph_set) return fail(s->err, SW_ESTATE, "node graph not set");
    if (!nbr8) return fail(s->err, SW_EINVAL, "NULL output");
    return guarded(s->err, [&]() -> sw_status {
        const int nn = s->h.nn;
        std::vector<int> lib((size_t)8 * nn);
        SWGN_HIP(hipMemcpyAsync(lib.data(), s->h.nbr, sizeof(int) * 8 * nn, hipMemcpyDeviceToHost, s->exec.st));
        SWGN_HIP(hipStreamSynchronize(s->exec.st));
        const std::vector<int>& pm = s->node_perm;
        for (int k = 0; k < nn; ++k)
            for (int q = 0; q < 8; ++q) nbr8[8 * (size_t)pm[k] + q] = pm[lib[8 * (size_t)k + q]];
        return SW_OK;
    });
}

sw_status sw_get_pattern(sw_stream s, int32_t* row_ptr, int32_t* col_idx) {
    if (!s) return SW_EINVAL;
    if (!s->graph_set) return fail(s->err, SW_ESTATE, "node graph not set");
    return guarded(s->err, [&]() -> sw_status {
        const CallerPattern cp = caller_pattern(s);
        if (row_ptr) std::memcpy(row_ptr, cp.row_ptr.data(), sizeof(int) * cp.row_ptr.size());
        if (col_idx) std::memcpy(col_idx, cp.col_idx.data(), sizeof(int) * cp.col_idx.size());
        return SW_OK;
    });
}

sw_status sw_get_last_maps(sw_stream s, int32_t* index_map, int32_t* corr_map, float* live_pos, float* depth_normals) {
    if (!s) return SW_EINVAL;
    if (s->server) server_quiesce(s->server, s);
    if (s->server && depth_normals)
        return fail(s->err, SW_ESTATE, "the normal map of an attached stream is not kept after its frame");
    if (!s->graph_set || !s->captured) return fail(s->err, SW_ESTATE, "no captured iteration");
    return guarded(s->err, [&]() -> sw_status {
        hipStream_t st = s->exec.st;
        const size_t npx = (size_t)s->h.npx;
        if (index_map) SWGN_HIP(hipMemcpyAsync(index_map, s->dbg_index, sizeof(int) * npx, hipMemcpyDeviceToHost, st));
        if (corr_map) SWGN_HIP(hipMemcpyAsync(corr_map, s->h.dbg_corr, sizeof(int) * npx, hipMemcpyDeviceToHost, st));
        if (live_pos) SWGN_HIP(hipMemcpyAsync(live_pos, s->h.dbg_live, sizeof(float) * 3 * s->ns, hipMemcpyDeviceToHost, st));
        std::vector<float4> nm;
        if (depth_normals) {
            nm.resize(npx);
            SWGN_HIP(hipMemcpyAsync(nm.data(), s->h.nmap, sizeof(float4) * npx, hipMemcpyDeviceToHost, st));
        }
        SWGN_HIP(hipStreamSynchronize(st));
        if (depth_normals) {
            for (size_t i = 0; i < npx; ++i) {
                depth_normals[i] = nm[i].x;
                depth_normals[npx + i] = nm[i].y;
                depth_normals[2 * npx + i] = nm[i].z;
            }
        }
        return SW_OK;
    });
}

sw_status sw_get_last_live_normals(sw_stream s, float* live_nrm) {
    if (!s || !live_nrm) return SW_EINVAL;
    if (s->server) server_quiesce(s->server, s);
    if (!s->graph_set || !s->captured) return fail(s->err, SW_ESTATE, "no captured iteration");
    return guarded(s->err, [&]() -> sw_status {
        hipStream_t st = s->exec.st;
        SWGN_HIP(hipMemcpyAsync(live_nrm, s->h.dbg_live + 3 * (size_t)s->ns, sizeof(float) * 3 * s->ns,
                                hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipStreamSynchronize(st));
        return SW_OK;
    });
}

sw_status sw_get_last_system(sw_stream s, float* blocks, float* g, float* delta) {
    if (!s) return SW_EINVAL;
    if (s->server) server_quiesce(s->server, s);
    if (!s->graph_set || !s->captured) return fail(s->err, SW_ESTATE, "no captured iteration");
    return guarded(s->err, [&]() -> sw_status {
        hipStream_t st = s->exec.st;
        const int nn = s->h.nn, nb = s->h.nb;
        std::vector<float> hb((size_t)36 * nb), hg((size_t)6 * nn), hx((size_t)6 * nn);
        SWGN_HIP(hipMemcpyAsync(hb.data(), s->dbg_H, sizeof(float) * 36 * nb, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipMemcpyAsync(hg.data(), s->dbg_g, sizeof(float) * 6 * nn, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipMemcpyAsync(hx.data(), s->dbg_x, sizeof(float) * 6 * nn, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipStreamSynchronize(st));
        // the caller's node order: node rows permuted, each upper block taken
        // from its library block, transposed where the two orders disagree
        const std::vector<int>& pm = s->node_perm;
        if (blocks) {
            const CallerPattern cp = caller_pattern(s);
            for (size_t b = 0; b < cp.src.size(); ++b) {
                const float* m = &hb[36 * (size_t)cp.src[b]];
                float* o = blocks + 36 * b;
                for (int r = 0; r < 6; ++r)
                    for (int c = 0; c < 6; ++c) o[6 * r + c] = cp.transposed[b] ? m[6 * c + r] : m[6 * r + c];
            }
        }
        for (int k = 0; k < nn; ++k) {
            if (g) std::memcpy(g + 6 * (size_t)pm[k], &hg[6 * (size_t)k], 6 * sizeof(float));
            if (delta) std::memcpy(delta + 6 * (size_t)pm[k], &hx[6 * (size_t)k], 6 * sizeof(float));
        }
        return SW_OK;
    });
}

sw_status sw_get_last_jacobian(sw_stream s, float* r, float* J) {
    if (!s) return SW_EINVAL;
    if (s->server) server_quiesce(s->server, s);
    if (!s->graph_set || !s->captured) return fail(s->err, SW_ESTATE, "no captured iteration");
    return guarded(s->err, [&]() -> sw_status {
        hipStream_t st = s->exec.st;
        const size_t ns = (size_t)s->ns, P = (size_t)s->h.pitch;
        std::vector<float> hJ(32 * P);
        std::vector<uint16_t> pos4(ns);
        std::vector<int> orig(ns);
        SWGN_HIP(hipMemcpyAsync(hJ.data(), s->dbg_J, sizeof(float) * 32 * P, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipMemcpyAsync(pos4.data(), s->h.pos4, sizeof(uint16_t) * ns, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipMemcpyAsync(orig.data(), s->h.orig, sizeof(int) * ns, hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipStreamSynchronize(st));
        for (size_t i = 0; i < ns; ++i) {
            const size_t o = (size_t)orig[i];
            const float* row = hJ.data() + 32 * i;
            if (r) r[o] = row[30];
            if (J) {
                for (int k = 0; k < 4; ++k) {
                    const int pos = (pos4[i] >> (3 * k)) & 7;
                    for (int c = 0; c < 6; ++c) J[24 * o + 6 * k + c] = row[pos * 6 + c];
                }
            }
        }
        return SW_OK;
    });
}

}  // extern "C"
