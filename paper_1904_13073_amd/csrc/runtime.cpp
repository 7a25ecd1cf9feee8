// C ABI of the swgn library: stream objects, device memory, the setup
// pipeline and the per-frame Gauss-Newton driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "swgn.h"
#include "swgn_impl.h"
#include "swgn_launch.h"

using namespace swgn;

namespace {

constexpr int kMaxIters = 16;
constexpr int kMaxPcg = 4096;
constexpr int kMaxNodes = 32768;
constexpr int64_t kMaxSurfels = (int64_t)1 << 28;

struct HipFail {
    hipError_t e;
    std::string what;
};

#define SWGN_HIP(x)                                                         \
    do {                                                                    \
        hipError_t _e = (x);                                                \
        if (_e != hipSuccess) throw HipFail{_e, std::string(#x)};           \
    } while (0)

// Device allocations released together.
class Arena {
public:
    ~Arena() { release(); }
    template <class T>
    T* alloc(size_t n) {
        void* p = nullptr;
        size_t bytes = (n == 0 ? 1 : n) * sizeof(T);
        bytes = (bytes + 255) & ~size_t(255);
        SWGN_HIP(hipMalloc(&p, bytes));
        ptrs_.push_back(p);
        return static_cast<T*>(p);
    }
    void release() {
        for (void* p : ptrs_) (void)hipFree(p);
        ptrs_.clear();
    }

private:
    std::vector<void*> ptrs_;
};

int pow2_at_least(int64_t n, int lo) {
    int64_t p = lo;
    while (p < n) p <<= 1;
    return (int)p;
}

bool finite(float v) { return std::isfinite(v); }

using IterStatsHost = IterStats;

}  // namespace

struct sw_stream_s {
    sw_config cfg{};
    hipStream_t st = nullptr;
    bool own_stream = false;
    std::string err;
    Cam cam{};

    Arena frame_mem, surf_mem, graph_mem;

    // per-image buffers
    float* depth = nullptr;
    float4* nmap = nullptr;
    unsigned long long* zbuf = nullptr;
    int* flags = nullptr;
    void* stats_d = nullptr;
    IterStatsHost* stats_h = nullptr;
    int* dbg_index = nullptr;
    int* dbg_corr = nullptr;

    // surfels as given
    int64_t ns = 0;
    float* in_pos = nullptr;
    float* in_nrm = nullptr;
    bool surfels_set = false;

    // node graph and everything derived from it
    bool graph_set = false;
    int nn = 0, nb = 0, nruns = 0, ne = 0, nf = 0, pitch = 0;
    float *spx, *spy, *spz, *snx, *sny, *snz;
    int4* sidx;
    float4* sw;
    int* sorig;
    float4 *pref, *rq, *tt, *dq, *cl, *rq_bak, *tt_bak;
    int* nbr;
    int *row_ptr, *col_idx, *blk_row;
    int ell_w = 0;
    uint32_t* ell_blk;
    int* ell_col;
    // assembly work lists: segments of surfels with one node set, per-block
    // (segment, positions) entries, node in-edges
    int* seg_start;
    int* ent_ptr;
    uint32_t* ent;
    int *in_ptr, *in_list;
    float* part;
    float *J, *H, *g, *ereg;
    double* Minv;
    double* part_e;
    int* part_n;
    float *x, *r, *z, *q, *p0, *p1;
    double *sc, *part_rho, *part_rr, *part_pq;
    int* offlist;
    // captured iteration
    float *dbg_live, *dbg_H, *dbg_g, *dbg_x, *dbg_J;
    bool captured = false;

    std::vector<hipEvent_t> events;

    ~sw_stream_s() {
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        if (stats_h) (void)hipHostFree(stats_h);
        graph_mem.release();
        surf_mem.release();
        frame_mem.release();
        if (own_stream && st) (void)hipStreamDestroy(st);
    }
};

namespace {

sw_status fail(sw_stream s, sw_status code, const std::string& msg) {
    if (s) s->err = msg;
    return code;
}

template <class F>
sw_status guarded(sw_stream s, F&& f) {
    try {
        return f();
    } catch (const HipFail& h) {
        sw_status code = (h.e == hipErrorOutOfMemory || h.e == hipErrorMemoryAllocation) ? SW_ENOMEM : SW_EHIP;
        return fail(s, code, h.what + ": " + hipGetErrorString(h.e));
    } catch (const std::bad_alloc&) {
        return fail(s, SW_ENOMEM, "host allocation failed");
    }
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
    if (c->jac_dtype != 0) { why = "jac_dtype: only 0 (fp32) is supported"; return SW_EINVAL; }
    if (c->dot_fp64 != 1) { why = "dot_fp64: PCG dot products accumulate in fp64 (1)"; return SW_EINVAL; }
    if (c->debug_iter < -1 || c->debug_iter >= kMaxIters) { why = "debug_iter out of range"; return SW_EINVAL; }
    if (c->stage_timing != 0 && c->stage_timing != 1) { why = "stage_timing must be 0 or 1"; return SW_EINVAL; }
    return SW_OK;
}

SurfelView surfel_view(const sw_stream_s* s) {
    return SurfelView{s->spx, s->spy, s->spz, s->snx, s->sny, s->snz, s->sidx, s->sw, s->sorig};
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

void build_graph(sw_stream s, int nn, const float* node_pos, const float* node_se3, int32_t on_device) {
    hipStream_t st = s->st;
    s->graph_mem.release();
    s->graph_set = false;
    s->captured = false;
    Arena tmp;
    Arena& G = s->graph_mem;
    const int ns = (int)s->ns;
    s->nn = nn;

    // nodes
    float* pos_in = tmp.alloc<float>(3 * (size_t)nn);
    copy_in(pos_in, node_pos, sizeof(float) * 3 * nn, on_device, st);
    s->pref = G.alloc<float4>(nn);
    launch_positions_to_f4(nn, pos_in, s->pref, st);
    s->rq = G.alloc<float4>(nn);
    s->tt = G.alloc<float4>(nn);
    s->dq = G.alloc<float4>(2 * (size_t)nn);
    s->cl = G.alloc<float4>(nn);
    s->rq_bak = G.alloc<float4>(nn);
    s->tt_bak = G.alloc<float4>(nn);
    float* se3_in = nullptr;
    if (node_se3) {
        se3_in = tmp.alloc<float>(12 * (size_t)nn);
        copy_in(se3_in, node_se3, sizeof(float) * 12 * nn, on_device, st);
    }
    launch_nodes_from_se3(nn, se3_in, s->pref, s->rq, s->tt, s->dq, s->cl, st);

    // skinning and node graph
    int4* idx_in = tmp.alloc<int4>(ns);
    float4* w_in = tmp.alloc<float4>(ns);
    float sig = s->cfg.node_sigma;
    launch_knn_skin(ns, s->in_pos, nn, s->pref, 1.0f / (2.0f * sig * sig), idx_in, w_in, st);
    s->nbr = G.alloc<int>(8 * (size_t)nn);
    launch_node_graph(nn, s->pref, s->nbr, st);

    // order surfels by node set
    int npad = pow2_at_least(ns, 1024);
    uint64_t* key = tmp.alloc<uint64_t>(npad);
    uint32_t* val = tmp.alloc<uint32_t>(npad);
    launch_tuple_keys(ns, npad, idx_in, key, val, st);
    sort_pairs(key, val, npad, st);
    s->pitch = (ns + 255) & ~255;
    s->spx = G.alloc<float>(s->pitch); s->spy = G.alloc<float>(s->pitch); s->spz = G.alloc<float>(s->pitch);
    s->snx = G.alloc<float>(s->pitch); s->sny = G.alloc<float>(s->pitch); s->snz = G.alloc<float>(s->pitch);
    s->sidx = G.alloc<int4>(s->pitch);
    s->sw = G.alloc<float4>(s->pitch);
    s->sorig = G.alloc<int>(s->pitch);
    int* flag = tmp.alloc<int>(ns + 1);
    int* fpos = tmp.alloc<int>(ns + 1);
    int* scan_tmp = tmp.alloc<int>(scan_tmp_size(std::max(10 * ns, 64 * nn) + 16));
    launch_permute_surfels(ns, kSegLen, key, val, s->in_pos, s->in_nrm, idx_in, w_in, s->spx, s->spy, s->spz, s->snx,
                           s->sny, s->snz, s->sidx, s->sw, s->sorig, flag, st);
    exclusive_scan(flag, fpos, ns, scan_tmp, st);
    s->nruns = read_scalar(fpos + ns, st);
    s->seg_start = G.alloc<int>(s->nruns + 1);
    int* run_start = s->seg_start;    // segments: ranges of one node set, at most kSegLen long
    launch_run_starts(ns, flag, fpos, run_start, st);

    // upper block pattern
    int words = (nn + 31) / 32;
    uint32_t* bm = tmp.alloc<uint32_t>((size_t)nn * words);
    launch_fill_i32(reinterpret_cast<int*>(bm), nn * words, 0, st);
    launch_pattern(s->nruns, key, run_start, nn, s->nbr, bm, words, st);
    int* rcnt = tmp.alloc<int>(nn);
    launch_row_counts(nn, bm, words, rcnt, st);
    s->row_ptr = G.alloc<int>(nn + 1);
    exclusive_scan(rcnt, s->row_ptr, nn, scan_tmp, st);
    s->nb = read_scalar(s->row_ptr + nn, st);
    s->col_idx = G.alloc<int>(s->nb);
    s->blk_row = G.alloc<int>(s->nb);
    launch_row_fill(nn, bm, words, s->row_ptr, s->col_idx, s->blk_row, st);

    // per-block run entries
    s->ne = 10 * s->nruns;
    int npad_e = pow2_at_least(s->ne, 1024);
    uint64_t* ekey = tmp.alloc<uint64_t>(npad_e);
    uint32_t* eval = tmp.alloc<uint32_t>(npad_e);
    int* ecount = tmp.alloc<int>(s->nb);
    launch_fill_i32(ecount, s->nb, 0, st);
    launch_run_entries(s->nruns, npad_e, key, run_start, s->row_ptr, s->col_idx, ekey, eval, ecount, st);
    sort_pairs(ekey, eval, npad_e, st);
    s->ent_ptr = G.alloc<int>(s->nb + 1);
    int* scan_tmp_b = tmp.alloc<int>(scan_tmp_size(std::max(s->nb, s->ne) + 16) + 16);
    exclusive_scan(ecount, s->ent_ptr, s->nb, scan_tmp_b, st);
    s->ent = G.alloc<uint32_t>(s->ne);
    launch_entries_store(s->ne, ekey, s->ent, st);
    const int noff = s->nb - nn;
    s->offlist = G.alloc<int>(std::max(1, noff));
    launch_offlist(s->nb, s->blk_row, s->col_idx, s->offlist, st);
    s->part = G.alloc<float>((size_t)kSegSlots * std::max(1, s->nruns));

    // in-edges of every node (j with the node in N_j), ascending j
    int npad_i = pow2_at_least(8 * (int64_t)nn, 1024);
    uint64_t* ikey = tmp.alloc<uint64_t>(npad_i);
    uint32_t* ival = tmp.alloc<uint32_t>(npad_i);
    int* icount = tmp.alloc<int>(nn);
    launch_fill_i32(icount, nn, 0, st);
    launch_in_edge_keys(nn, npad_i, s->nbr, ikey, ival, icount, st);
    sort_pairs(ikey, ival, npad_i, st);
    s->in_ptr = G.alloc<int>(nn + 1);
    exclusive_scan(icount, s->in_ptr, nn, scan_tmp, st);
    s->in_list = G.alloc<int>(8 * (size_t)nn);
    launch_in_edge_store(8 * nn, ival, s->in_list, st);

    // full symmetric rows for the matrix product
    int npad_t = pow2_at_least(s->nb, 1024);
    uint64_t* tkey = tmp.alloc<uint64_t>(npad_t);
    uint32_t* tval = tmp.alloc<uint32_t>(npad_t);
    int* tcount = tmp.alloc<int>(nn);
    launch_fill_i32(tcount, nn, 0, st);
    launch_transpose_keys(s->nb, npad_t, s->blk_row, s->col_idx, tkey, tval, tcount, st);
    sort_pairs(tkey, tval, npad_t, st);
    int* tstart = tmp.alloc<int>(nn + 1);
    exclusive_scan(tcount, tstart, nn, scan_tmp, st);
    int* fcount = tmp.alloc<int>(nn);
    launch_full_counts(nn, s->row_ptr, tcount, fcount, st);
    int* frow_ptr = tmp.alloc<int>(nn + 1);
    exclusive_scan(fcount, frow_ptr, nn, scan_tmp, st);
    s->nf = 2 * s->nb - nn;
    uint32_t* fblk = tmp.alloc<uint32_t>(s->nf);
    int* fcol = tmp.alloc<int>(s->nf);
    launch_full_rows(nn, s->nb - nn, s->row_ptr, s->col_idx, tcount, tstart, frow_ptr, tkey, tval, fblk, fcol, st);
    {
        std::vector<int> hrow(nn + 1);
        SWGN_HIP(hipMemcpyAsync(hrow.data(), frow_ptr, sizeof(int) * (nn + 1), hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipStreamSynchronize(st));
        int wmax = 1;
        for (int k = 0; k < nn; ++k) wmax = std::max(wmax, hrow[k + 1] - hrow[k]);
        s->ell_w = (wmax + 7) & ~7;
    }
    s->ell_blk = G.alloc<uint32_t>((size_t)nn * s->ell_w);
    s->ell_col = G.alloc<int>((size_t)nn * s->ell_w);
    launch_ell(nn, s->ell_w, frow_ptr, fblk, fcol, s->ell_blk, s->ell_col, st);

    // per-iteration buffers
    s->J = G.alloc<float>(32 * (size_t)s->pitch);
    launch_fill_i32(reinterpret_cast<int*>(s->J), 32 * s->pitch, 0, st);   // padding columns stay zero
    s->H = G.alloc<float>(36 * (size_t)s->nb);
    s->g = G.alloc<float>(6 * (size_t)nn);
    s->ereg = G.alloc<float>(nn);
    s->Minv = G.alloc<double>(36 * (size_t)nn);
    int ncb = corr_blocks(ns);
    s->part_e = G.alloc<double>(ncb);
    s->part_n = G.alloc<int>(ncb);
    size_t n6 = 6 * (size_t)nn;
    s->x = G.alloc<float>(n6); s->r = G.alloc<float>(n6); s->z = G.alloc<float>(n6); s->q = G.alloc<float>(n6);
    s->p0 = G.alloc<float>(n6); s->p1 = G.alloc<float>(n6);
    const int nparts = solve_partials_size(nn);
    s->sc = G.alloc<double>(2 * (kMaxPcg + 1));
    s->part_rho = G.alloc<double>(nparts);
    s->part_rr = G.alloc<double>(nparts);
    s->part_pq = G.alloc<double>(nparts);
    s->dbg_live = G.alloc<float>(3 * (size_t)ns);
    s->dbg_H = G.alloc<float>(36 * (size_t)s->nb);
    s->dbg_g = G.alloc<float>(n6);
    s->dbg_x = G.alloc<float>(n6);
    s->dbg_J = G.alloc<float>(32 * (size_t)s->pitch);

    SWGN_HIP(hipGetLastError());
    SWGN_HIP(hipStreamSynchronize(st));
    s->graph_set = true;
}

hipEvent_t event_at(sw_stream s, size_t i) {
    while (s->events.size() <= i) {
        hipEvent_t e;
        SWGN_HIP(hipEventCreate(&e));
        s->events.push_back(e);
    }
    return s->events[i];
}

double model_bytes(const sw_stream_s* s, int64_t n_corr_total) {
    // algorithmic bytes of one frame: data each kernel must read or write at least
    double ns = (double)s->ns, nn = (double)s->nn, nb = (double)s->nb;
    double npx = (double)s->cam.W * s->cam.H;
    double per_iter = 0.0;
    per_iter += 48.0 * ns + 8.0 * ns + 8.0 * npx;                 // warp + z-buffer (+ clear)
    per_iter += 60.0 * ns + 8.0 * ns + 16.0 * ns + 100.0 * ns;    // correspondence + J
    per_iter += 2.0 * kSegSlots * 4.0 * s->nruns + 144.0 * nb + 24.0 * nn;  // segment Grams + blocks
    per_iter += 144.0 * nn + 288.0 * nn;                          // block-Jacobi
    per_iter += s->cfg.pcg_iters * (144.0 * nb + 7.0 * 24.0 * nn); // PCG
    double frame = s->cfg.gn_iters * per_iter + 20.0 * npx;
    frame += 100.0 * (double)n_corr_total;                        // J read by the assembly
    return frame;
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
    sw_status rc = guarded(s, [&]() -> sw_status {
        s->cfg = *cfg;
        s->cam = Cam{cfg->width, cfg->height, cfg->fx, cfg->fy, cfg->cx, cfg->cy};
        if (hip_stream) {
            s->st = static_cast<hipStream_t>(hip_stream);
        } else {
            SWGN_HIP(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking));
            s->own_stream = true;
        }
        size_t npx = (size_t)cfg->width * cfg->height;
        s->depth = s->frame_mem.alloc<float>(npx);
        s->nmap = s->frame_mem.alloc<float4>(npx);
        s->zbuf = s->frame_mem.alloc<unsigned long long>(npx);
        s->dbg_index = s->frame_mem.alloc<int>(npx);
        s->dbg_corr = s->frame_mem.alloc<int>(npx);
        s->flags = s->frame_mem.alloc<int>(4);
        s->stats_d = s->frame_mem.alloc<char>(sizeof(IterStats) * kMaxIters);
        void* h = nullptr;
        SWGN_HIP(hipHostMalloc(&h, sizeof(IterStatsHost) * kMaxIters + 64, hipHostMallocDefault));
        s->stats_h = static_cast<IterStatsHost*>(h);
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
    if (s->st) (void)hipStreamSynchronize(s->st);
    delete s;
    return SW_OK;
}

sw_status sw_set_reference_surfels(sw_stream s, int64_t n, const float* pos, const float* nrm, int32_t on_device) {
    if (!s) return SW_EINVAL;
    if (n < 1 || n >= kMaxSurfels) return fail(s, SW_EINVAL, "surfel count out of range");
    if (!pos || !nrm) return fail(s, SW_EINVAL, "surfel pointers must not be NULL");
    if (on_device != 0 && on_device != 1) return fail(s, SW_EINVAL, "on_device must be 0 or 1");
    return guarded(s, [&]() -> sw_status {
        s->graph_mem.release();
        s->graph_set = false;
        s->captured = false;
        s->surf_mem.release();
        s->surfels_set = false;
        s->ns = n;
        s->in_pos = s->surf_mem.alloc<float>(3 * (size_t)n);
        s->in_nrm = s->surf_mem.alloc<float>(3 * (size_t)n);
        copy_in(s->in_pos, pos, sizeof(float) * 3 * n, on_device, s->st);
        copy_in(s->in_nrm, nrm, sizeof(float) * 3 * n, on_device, s->st);
        SWGN_HIP(hipStreamSynchronize(s->st));
        s->surfels_set = true;
        return SW_OK;
    });
}

sw_status sw_set_node_graph(sw_stream s, int32_t n_nodes, const float* node_pos, const float* node_se3,
                            int32_t on_device) {
    if (!s) return SW_EINVAL;
    if (!s->surfels_set) return fail(s, SW_ESTATE, "reference surfels must be set before the node graph");
    if (n_nodes < 9 || n_nodes > kMaxNodes) return fail(s, SW_EINVAL, "n_nodes must be in [9, 32768]");
    if (!node_pos) return fail(s, SW_EINVAL, "node positions must not be NULL");
    if (on_device != 0 && on_device != 1) return fail(s, SW_EINVAL, "on_device must be 0 or 1");
    return guarded(s, [&]() -> sw_status {
        build_graph(s, n_nodes, node_pos, node_se3, on_device);
        return SW_OK;
    });
}

sw_status sw_set_node_se3(sw_stream s, const float* node_se3, int32_t n, int32_t on_device) {
    if (!s) return SW_EINVAL;
    if (!s->graph_set) return fail(s, SW_ESTATE, "node graph not set");
    if (n != s->nn || !node_se3) return fail(s, SW_EINVAL, "need n_nodes transforms");
    if (on_device != 0 && on_device != 1) return fail(s, SW_EINVAL, "on_device must be 0 or 1");
    return guarded(s, [&]() -> sw_status {
        Arena tmp;
        float* d = tmp.alloc<float>(12 * (size_t)n);
        copy_in(d, node_se3, sizeof(float) * 12 * n, on_device, s->st);
        launch_nodes_from_se3(n, d, s->pref, s->rq, s->tt, s->dq, s->cl, s->st);
        SWGN_HIP(hipGetLastError());
        SWGN_HIP(hipStreamSynchronize(s->st));
        return SW_OK;
    });
}

sw_status sw_solve_frame(sw_stream s, const float* depth, int32_t on_device, sw_frame_stats* stats) {
    if (!s) return SW_EINVAL;
    if (!s->graph_set) return fail(s, SW_ESTATE, "surfels and node graph must be set before solving");
    if (!depth) return fail(s, SW_EINVAL, "depth must not be NULL");
    if (on_device != 0 && on_device != 1) return fail(s, SW_EINVAL, "on_device must be 0 or 1");
    return guarded(s, [&]() -> sw_status {
        hipStream_t st = s->st;
        const sw_config& c = s->cfg;
        const int ns = (int)s->ns, nn = s->nn;
        const int npx = s->cam.W * s->cam.H;
        const bool timing = c.stage_timing != 0;
        size_t ev = 0;
        std::vector<int> ev_kernel;
        auto mark = [&](int kernel) {
            if (!timing) return;
            SWGN_HIP(hipEventRecord(event_at(s, ev++), st));
            ev_kernel.push_back(kernel);
        };
        const float* d = depth;
        if (!on_device) {
            copy_in(s->depth, depth, sizeof(float) * npx, 0, st);
            d = s->depth;
        }
        SWGN_HIP(hipMemcpyAsync(s->rq_bak, s->rq, sizeof(float4) * nn, hipMemcpyDeviceToDevice, st));
        SWGN_HIP(hipMemcpyAsync(s->tt_bak, s->tt, sizeof(float4) * nn, hipMemcpyDeviceToDevice, st));
        mark(0);
        launch_depth_prep(s->cam, d, c.edge_gate, s->nmap, s->zbuf, s->flags, st);
        mark(-1);
        const SurfelView sv = surfel_view(s);
        const float dist2 = c.corr_dist * c.corr_dist;
        char* stats_d = static_cast<char*>(s->stats_d);
        const size_t iss = sizeof(IterStats);
        AssembleArgs aa{s->nb, nn, s->nb - nn, s->pitch, s->nruns, s->blk_row, s->col_idx, s->row_ptr,
                        s->offlist, s->seg_start, s->ent_ptr, s->ent, s->in_ptr, s->in_list, s->J, s->nbr,
                        s->pref, s->rq, s->cl, c.lambda_reg, c.damping, s->part, s->H, s->g, s->ereg};
        SolveStepArgs sa{nn, npx, s->row_ptr, s->H, s->g, s->ell_w, s->ell_blk, s->ell_col, s->Minv,
                         s->x, s->r, s->z, s->q, s->p0, s->p1, s->sc, s->part_rho, s->part_rr, s->part_pq, s->flags,
                         s->part_e, s->part_n, corr_blocks(ns), s->ereg, nullptr, s->pref, s->rq, s->tt, s->dq,
                         s->cl, s->zbuf};
        bool capture_done = false;
        for (int it = 0; it < c.gn_iters; ++it) {
            const bool cap = (it == c.debug_iter);
            mark(1);
            launch_warp_zbuf(ns, sv, s->dq, s->cam, s->zbuf, st);
            mark(-1);
            if (cap) {
                launch_export_index_map(npx, s->zbuf, s->dbg_index, st);
                launch_fill_i32(s->dbg_corr, npx, -1, st);
            }
            mark(2);
            launch_corr_jac(ns, sv, s->dq, s->cl, s->cam, s->zbuf, s->nmap, dist2, c.corr_normal, s->J,
                            s->pitch, s->part_e, s->part_n, cap ? s->dbg_corr : nullptr,
                            cap ? s->dbg_live : nullptr, st);
            mark(-1);
            mark(3);
            launch_assemble_segments(aa, st);
            mark(-1);
            mark(8);
            launch_assemble_fold(aa, st);
            mark(-1);
            if (cap) {
                // the solve step updates the node state: keep this iteration's system first
                SWGN_HIP(hipMemcpyAsync(s->dbg_J, s->J, sizeof(float) * 32 * s->pitch, hipMemcpyDeviceToDevice, st));
                SWGN_HIP(hipMemcpyAsync(s->dbg_H, s->H, sizeof(float) * 36 * s->nb, hipMemcpyDeviceToDevice, st));
                SWGN_HIP(hipMemcpyAsync(s->dbg_g, s->g, sizeof(float) * 6 * nn, hipMemcpyDeviceToDevice, st));
            }
            sa.stats = stats_d + iss * it;
            mark(4);
            launch_pcg_init(sa, st);
            mark(-1);
            for (int pit = 0; pit < c.pcg_iters; ++pit) {
                mark(5);
                launch_pcg_spmv(sa, pit, st);
                mark(-1);
                mark(6);
                launch_pcg_update(sa, pit, st);
                mark(-1);
            }
            mark(7);
            launch_node_update(sa, c.pcg_iters, st);
            mark(-1);
            if (cap) {
                SWGN_HIP(hipMemcpyAsync(s->dbg_x, s->x, sizeof(float) * 6 * nn, hipMemcpyDeviceToDevice, st));
                capture_done = true;
            }
        }
        SWGN_HIP(hipGetLastError());
        const int G = c.gn_iters;
        if (G > 0)
            SWGN_HIP(hipMemcpyAsync(s->stats_h, s->stats_d, iss * G, hipMemcpyDeviceToHost, st));
        int* hflags = reinterpret_cast<int*>(reinterpret_cast<char*>(s->stats_h) + sizeof(IterStatsHost) * kMaxIters);
        SWGN_HIP(hipMemcpyAsync(hflags, s->flags, sizeof(int), hipMemcpyDeviceToHost, st));
        SWGN_HIP(hipStreamSynchronize(st));
        if (capture_done) s->captured = true;
        int64_t ncorr_total = 0;
        bool bad = (*hflags != 0);
        for (int it = 0; it < G; ++it) {
            const IterStatsHost& h = s->stats_h[it];
            ncorr_total += h.n_corr;
            if (!std::isfinite(h.e_data) || !std::isfinite(h.e_reg)) bad = true;
        }
        if (stats) {
            std::memset(stats, 0, sizeof(*stats));
            stats->iters = G;
            for (int it = 0; it < G; ++it) {
                const IterStatsHost& h = s->stats_h[it];
                stats->e_data[it] = (float)h.e_data;
                stats->e_reg[it] = (float)h.e_reg;
                stats->n_corr[it] = h.n_corr;
                stats->pcg_resid[it] = (float)h.pcg_resid;
            }
            if (timing) {
                // events come in (start of kernel id, end) pairs
                for (size_t a = 0; a + 1 < ev; a += 2) {
                    float ms = 0.f;
                    SWGN_HIP(hipEventElapsedTime(&ms, s->events[a], s->events[a + 1]));
                    stats->stage_us[ev_kernel[a]] += 1000.f * ms;
                }
            }
            stats->alg_bytes = model_bytes(s, ncorr_total);
        }
        if (bad) {
            SWGN_HIP(hipMemcpyAsync(s->rq, s->rq_bak, sizeof(float4) * nn, hipMemcpyDeviceToDevice, st));
            SWGN_HIP(hipMemcpyAsync(s->tt, s->tt_bak, sizeof(float4) * nn, hipMemcpyDeviceToDevice, st));
            launch_tables_from_state(nn, s->pref, s->rq, s->tt, s->dq, s->cl, st);
            SWGN_HIP(hipStreamSynchronize(st));
            return fail(s, SW_ENUMERIC, "non-finite energy, node update or non-positive-definite diagonal block;"
                                        " node transforms restored");
        }
        return SW_OK;
    });
}

sw_status sw_get_node_se3(sw_stream s, float* out, int32_t capacity) {
    if (!s) return SW_EINVAL;
    if (!s->graph_set) return fail(s, SW_ESTATE, "node graph not set");
    if (!out || capacity < s->nn) return fail(s, SW_EINVAL, "output capacity below n_nodes");
    return guarded(s, [&]() -> sw_status {
        Arena tmp;
        float* d = tmp.alloc<float>(12 * (size_t)s->nn);
        launch_node_se3_out(s->nn, s->rq, s->tt, d, s->st);
        SWGN_HIP(hipMemcpyAsync(out, d, sizeof(float) * 12 * s->nn, hipMemcpyDeviceToHost, s->st));
        SWGN_HIP(hipStreamSynchronize(s->st));
        return SW_OK;
    });
}

sw_status sw_get_sizes(sw_stream s, int64_t* n_surfels, int32_t* n_nodes, int32_t* n_blocks) {
    if (!s) return SW_EINVAL;
    if (n_surfels) *n_surfels = s->ns;
    if (n_nodes) *n_nodes = s->graph_set ? s->nn : 0;
    if (n_blocks) *n_blocks = s->graph_set ? s->nb : 0;
    return SW_OK;
}

sw_status sw_get_skinning(sw_stream s, int32_t* idx4, float* w4) {
    if (!s) return SW_EINVAL;
    if (!s->graph_set) return fail(s, SW_ESTATE, "node graph not set");
    return guarded(s, [&]() -> sw_status {
        const size_t ns = (size_t)s->ns;
        std::vector<int4> idx(ns);
        std::vector<float4> w(ns);
        std::vector<int> orig(ns);
        SWGN_HIP(hipMemcpyAsync(idx.data(), s->sidx, sizeof(int4) * ns, hipMemcpyDeviceToHost, s->st));
        SWGN_HIP(hipMemcpyAsync(w.data(), s->sw, sizeof(float4) * ns, hipMemcpyDeviceToHost, s->st));
        SWGN_HIP(hipMemcpyAsync(orig.data(), s->sorig, sizeof(int) * ns, hipMemcpyDeviceToHost, s->st));
        SWGN_HIP(hipStreamSynchronize(s->st));
        for (size_t i = 0; i < ns; ++i) {
            size_t o = (size_t)orig[i];
            if (idx4) { idx4[4 * o] = idx[i].x; idx4[4 * o + 1] = idx[i].y; idx4[4 * o + 2] = idx[i].z; idx4[4 * o + 3] = idx[i].w; }
            if (w4) { w4[4 * o] = w[i].x; w4[4 * o + 1] = w[i].y; w4[4 * o + 2] = w[i].z; w4[4 * o + 3] = w[i].w; }
        }
        return SW_OK;
    });
}

sw_status sw_get_node_graph(sw_stream s, int32_t* nbr8) {
    if (!s) return SW_EINVAL;
    if (!s->graph_set) return fail(s, SW_ESTATE, "node graph not set");
    if (!nbr8) return fail(s, SW_EINVAL, "NULL output");
    return guarded(s, [&]() -> sw_status {
        SWGN_HIP(hipMemcpyAsync(nbr8, s->nbr, sizeof(int) * 8 * s->nn, hipMemcpyDeviceToHost, s->st));
        SWGN_HIP(hipStreamSynchronize(s->st));
        return SW_OK;
    });
}

sw_status sw_get_pattern(sw_stream s, int32_t* row_ptr, int32_t* col_idx) {
    if (!s) return SW_EINVAL;
    if (!s->graph_set) return fail(s, SW_ESTATE, "node graph not set");
    return guarded(s, [&]() -> sw_status {
        if (row_ptr) SWGN_HIP(hipMemcpyAsync(row_ptr, s->row_ptr, sizeof(int) * (s->nn + 1), hipMemcpyDeviceToHost, s->st));
        if (col_idx) SWGN_HIP(hipMemcpyAsync(col_idx, s->col_idx, sizeof(int) * s->nb, hipMemcpyDeviceToHost, s->st));
        SWGN_HIP(hipStreamSynchronize(s->st));
        return SW_OK;
    });
}

sw_status sw_get_last_maps(sw_stream s, int32_t* index_map, int32_t* corr_map, float* live_pos, float* depth_normals) {
    if (!s) return SW_EINVAL;
    if (!s->graph_set || !s->captured) return fail(s, SW_ESTATE, "no captured iteration");
    return guarded(s, [&]() -> sw_status {
        const size_t npx = (size_t)s->cam.W * s->cam.H;
        if (index_map) SWGN_HIP(hipMemcpyAsync(index_map, s->dbg_index, sizeof(int) * npx, hipMemcpyDeviceToHost, s->st));
        if (corr_map) SWGN_HIP(hipMemcpyAsync(corr_map, s->dbg_corr, sizeof(int) * npx, hipMemcpyDeviceToHost, s->st));
        if (live_pos) SWGN_HIP(hipMemcpyAsync(live_pos, s->dbg_live, sizeof(float) * 3 * s->ns, hipMemcpyDeviceToHost, s->st));
        std::vector<float4> nm;
        if (depth_normals) {
            nm.resize(npx);
            SWGN_HIP(hipMemcpyAsync(nm.data(), s->nmap, sizeof(float4) * npx, hipMemcpyDeviceToHost, s->st));
        }
        SWGN_HIP(hipStreamSynchronize(s->st));
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

sw_status sw_get_last_system(sw_stream s, float* blocks, float* g, float* delta) {
    if (!s) return SW_EINVAL;
    if (!s->graph_set || !s->captured) return fail(s, SW_ESTATE, "no captured iteration");
    return guarded(s, [&]() -> sw_status {
        if (blocks) SWGN_HIP(hipMemcpyAsync(blocks, s->dbg_H, sizeof(float) * 36 * s->nb, hipMemcpyDeviceToHost, s->st));
        if (g) SWGN_HIP(hipMemcpyAsync(g, s->dbg_g, sizeof(float) * 6 * s->nn, hipMemcpyDeviceToHost, s->st));
        if (delta) SWGN_HIP(hipMemcpyAsync(delta, s->dbg_x, sizeof(float) * 6 * s->nn, hipMemcpyDeviceToHost, s->st));
        SWGN_HIP(hipStreamSynchronize(s->st));
        return SW_OK;
    });
}

sw_status sw_get_last_jacobian(sw_stream s, float* r, float* J) {
    if (!s) return SW_EINVAL;
    if (!s->graph_set || !s->captured) return fail(s, SW_ESTATE, "no captured iteration");
    return guarded(s, [&]() -> sw_status {
        const size_t ns = (size_t)s->ns, P = (size_t)s->pitch;
        std::vector<float> hJ(32 * P);
        std::vector<int4> idx(ns);
        std::vector<int> orig(ns);
        SWGN_HIP(hipMemcpyAsync(hJ.data(), s->dbg_J, sizeof(float) * 32 * P, hipMemcpyDeviceToHost, s->st));
        SWGN_HIP(hipMemcpyAsync(idx.data(), s->sidx, sizeof(int4) * ns, hipMemcpyDeviceToHost, s->st));
        SWGN_HIP(hipMemcpyAsync(orig.data(), s->sorig, sizeof(int) * ns, hipMemcpyDeviceToHost, s->st));
        SWGN_HIP(hipStreamSynchronize(s->st));
        for (size_t i = 0; i < ns; ++i) {
            const size_t o = (size_t)orig[i];
            const float* row = hJ.data() + 32 * i;
            if (r) r[o] = row[24];
            if (J) {
                const int ids[4] = {idx[i].x, idx[i].y, idx[i].z, idx[i].w};
                for (int k = 0; k < 4; ++k) {
                    int pos = (ids[0] < ids[k]) + (ids[1] < ids[k]) + (ids[2] < ids[k]) + (ids[3] < ids[k]);
                    for (int c = 0; c < 6; ++c) J[24 * o + 6 * k + c] = row[pos * 6 + c];
                }
            }
        }
        return SW_OK;
    });
}

}  // extern "C"
