// Host-side objects shared by the C ABI files: device arenas, executors (a
// HIP stream with its statistics buffers and timing events) and the stream
// object itself.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <utility>
#include <string>
#include <vector>

#include "swgn.h"
#include "swgn_frame.h"

namespace swgn {
namespace rt {

constexpr int kMaxNodes = 32768;
// Untuned batches take fused PCG steps up to this many rows in all (where one
// launch per iteration beats two; above it the products' re-reads cost more).
constexpr int64_t kFusedRows = 8192;
constexpr int kPcgAuto = 0, kPcgSplit = 1, kPcgFused = 2;
constexpr int64_t kMaxSurfels = (int64_t)1 << 28;

struct HipFail {
    hipError_t e;
    std::string what;
};

#define SWGN_HIP(x)                                                         \
    do {                                                                    \
        hipError_t _e = (x);                                                \
        if (_e != hipSuccess) throw ::swgn::rt::HipFail{_e, std::string(#x)}; \
    } while (0)

// Device allocations released together.
class Arena {
public:
    ~Arena() { release(); }
    // 256-byte aligned; carved from the current chunk of device memory or a new
    // one (chunks grow geometrically from 4 MiB, so an arena of many arrays
    // costs a few hipMalloc calls, not one per array)
    void* raw(size_t bytes);
    template <class T>
    T* alloc(size_t n) {
        return static_cast<T*>(raw(n * sizeof(T)));
    }
    void release();
    // hands the chunks out again from the start (no device memory is freed;
    // the caller makes sure no work still uses what they held)
    void reset();
    size_t bytes() const { return bytes_; }   // bytes handed out (aligned)
    void swap(Arena& o) {
        chunks_.swap(o.chunks_);
        std::swap(cur_, o.cur_);
        std::swap(bytes_, o.bytes_);
    }

private:
    struct Chunk {
        char* base;
        size_t size, used;
    };
    std::vector<Chunk> chunks_;
    size_t cur_ = 0;                      // chunk handed out from
    size_t bytes_ = 0;
};

// A HIP stream plus what a solve needs besides the streams' own memory: the
// device and pinned host slots of the statistics copy (kMaxBatch streams)
// and timing events.
struct Executor {
    hipStream_t st = nullptr;
    bool own_stream = false;
    char* stats_dev = nullptr;
    void* stats_host = nullptr;
    std::vector<hipEvent_t> events;
    // launch variant per stage (kVarXcd | kVarWide bits), per shape bucket of
    // a batch; chosen by the autotuner, a size rule where it has not run
    std::map<uint64_t, std::vector<int>> tuned;
    uint64_t bucket = 0;                  // bucket of the batch being launched
    uint64_t tune_epoch = 0;              // bumped when a choice changes (captured graphs are stale)
    int variant_of(int stage, int64_t rows) const;
    // replay of a batch's iterations as one HIP graph
    bool graphs = false;
    int pcg_mode = 0;                     // kPcgAuto, kPcgSplit, kPcgFused
    hipGraphExec_t graph_exec = nullptr;
    std::vector<std::pair<sw_stream, uint64_t>> graph_key;   // (stream, generation) it was captured for
    ~Executor();
    void init(void* hip_stream);
    hipEvent_t event(size_t i);
    void drop_graph();
};

inline sw_status fail(std::string& err, sw_status code, const std::string& msg) {
    err = msg;
    return code;
}

template <class F>
sw_status guarded(std::string& err, F&& f) {
    try {
        return f();
    } catch (const HipFail& h) {
        const sw_status code =
            (h.e == hipErrorOutOfMemory || h.e == hipErrorMemoryAllocation) ? SW_ENOMEM : SW_EHIP;
        return fail(err, code, h.what + ": " + hipGetErrorString(h.e));
    } catch (const std::bad_alloc&) {
        return fail(err, SW_ENOMEM, "host allocation failed");
    }
}

size_t carve_workspace(FrameDesc& h, char* base);

}  // namespace rt
}  // namespace swgn

struct sw_stream_s {
    sw_config cfg{};
    swgn::Cam cam{};
    std::string err;
    swgn::rt::Executor exec;              // the stream's own HIP stream
    swgn::rt::Arena frame_mem, surf_mem, graph_mem, ws_mem;
    swgn::rt::Arena setup_mem;            // temporaries of the node-set build, kept for the next one
    uint64_t generation = 0;              // bumped whenever device buffers are replaced

    // surfels as given
    int64_t ns = 0;
    float* in_pos = nullptr;
    float* in_nrm = nullptr;
    float* in_rad = nullptr;              // attributes, caller order (kept current by fusion)
    float* in_conf = nullptr;
    int* in_tobs = nullptr;
    int* in_tinit = nullptr;
    int t_now = 0;                        // frame time (visibility of recent surfels)

    // depth-map fusion workspace, allocated on first use
    swgn::rt::Arena fuse_mem;
    unsigned long long* fz4 = nullptr;    // 4x super-sampled index map
    float* flive = nullptr;               // [6][pitch] live positions and normals of the last fusion
    int* fmatch = nullptr;                // [npx]
    int* fcount = nullptr;                // [2]
    int* fcount_host = nullptr;           // pinned, [8]: fusion counts, append counts
    bool fused = false;
    uint64_t depth_gen = 0;               // bumped by every depth preprocessing
    uint64_t fuse_gen = ~0ull;            // depth_gen of the last fusion
    // append-candidate workspace, allocated on first use
    swgn::rt::Arena append_mem;
    int *aflag = nullptr, *apos = nullptr, *ascan = nullptr, *acount = nullptr;
    float4 *asv = nullptr, *asn = nullptr;
    int* apix = nullptr;                  // staging of host outputs, capacity npx
    float *apos3 = nullptr, *anrm3 = nullptr, *arad = nullptr, *aconf = nullptr;
    bool surfels_set = false;
    bool graph_set = false;
    sw_server server = nullptr;           // set while attached to a serving loop

    // descriptor: host copy, pinned staging copy and the device copy kernels read
    swgn::FrameDesc h{};
    swgn::FrameDesc* h_pinned = nullptr;
    swgn::FrameDesc* d_desc = nullptr;
    size_t ws_bytes = 0;
    int nsets = 0;                        // distinct node sets
    int64_t nent = 0;                     // block-fold entries

    // node numbering: the library keeps nodes in a spatially local order
    // (Morton order of their reference positions), so that a block row's
    // columns lie near it; every export is in the caller's order
    std::vector<int> node_perm;           // library index k -> caller index
    std::vector<int> node_inv;            // caller index -> library index
    int* d_node_id = nullptr;             // [nn] node_perm on the device
    int* d_node_inv = nullptr;            // [nn] node_inv on the device

    // captured iteration (allocated only when the config asks for a capture)
    int* dbg_index = nullptr;
    float *dbg_H = nullptr, *dbg_g = nullptr, *dbg_x = nullptr, *dbg_J = nullptr;
    bool captured = false;

    ~sw_stream_s() {
        if (h_pinned) (void)hipHostFree(h_pinned);
        if (fcount_host) (void)hipHostFree(fcount_host);
    }
};

namespace swgn {
namespace rt {
// update: a PCG finish or fused step launch that also performs the node
// update of every stream whose last finish it holds (not for replays)
void run_stage(Executor& ex, int stage, const std::vector<sw_stream>& ss, const std::vector<int>& its, int pcg_it,
               const DepthIn* depth, bool timing, std::vector<int>& ev_stage, bool update = false);
void enqueue_depth(Executor& ex, const std::vector<sw_stream>& ss, const float* const* depths, int32_t on_device,
                   bool timing, std::vector<int>& ev);
void enqueue_rigid(Executor& ex, const std::vector<sw_stream>& ss, bool timing, std::vector<int>& ev);
void enqueue_iteration(Executor& ex, const std::vector<sw_stream>& ss, const std::vector<int>& its, bool timing,
                       std::vector<int>& ev, std::vector<char>& captured);
void enqueue_collect(Executor& ex, const std::vector<sw_stream>& ss);
sw_status collect_frames(Executor& ex, const std::vector<sw_stream>& ss, const float* stage_us,
                         sw_frame_stats* stats, sw_status* status);
sw_status finish_frames(Executor& ex, const std::vector<sw_stream>& ss, const float* stage_us,
                        sw_frame_stats* stats, sw_status* status);
uint64_t shape_bucket(const std::vector<sw_stream>& ss);
void server_quiesce(sw_server sv, sw_stream s);
void server_forget(sw_server sv, sw_stream s);
sw_status solve_frames(Executor& ex, const std::vector<sw_stream>& ss, const float* const* depths,
                       int32_t on_device, bool timing, sw_frame_stats* stats, sw_status* status);
}  // namespace rt
}  // namespace swgn
