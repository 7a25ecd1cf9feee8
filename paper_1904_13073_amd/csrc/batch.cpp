// C ABI of batched solves: one frame for each of several streams, with one
// launch per Gauss-Newton stage covering all of them (the streams' tiles
// concatenated in one grid, see swgn_frame.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "runtime_internal.h"
#include "swgn.h"
#include "swgn_frame.h"

using namespace swgn;
using namespace swgn::rt;

struct sw_batch_s {
    Executor exec;
    std::string err;
    int32_t flags = 0;
};

extern "C" {

sw_status sw_create_batch(void* hip_stream, int32_t flags, sw_batch* out) {
    if (!out) return SW_EINVAL;
    *out = nullptr;
    if (flags & ~(SW_BATCH_TIMING | SW_BATCH_GRAPH | SW_BATCH_PCG_SPLIT | SW_BATCH_PCG_FUSED)) return SW_EINVAL;
    if ((flags & SW_BATCH_TIMING) && (flags & SW_BATCH_GRAPH)) return SW_EINVAL;
    if ((flags & SW_BATCH_PCG_SPLIT) && (flags & SW_BATCH_PCG_FUSED)) return SW_EINVAL;
    sw_batch_s* b = new (std::nothrow) sw_batch_s();
    if (!b) return SW_ENOMEM;
    const sw_status rc = guarded(b->err, [&]() -> sw_status {
        b->flags = flags;
        b->exec.init(hip_stream);
        b->exec.graphs = (flags & SW_BATCH_GRAPH) != 0;
        b->exec.pcg_mode = (flags & SW_BATCH_PCG_SPLIT) ? kPcgSplit : (flags & SW_BATCH_PCG_FUSED) ? kPcgFused : kPcgAuto;
        return SW_OK;
    });
    if (rc != SW_OK) {
        delete b;
        return rc;
    }
    *out = b;
    return SW_OK;
}

sw_status sw_destroy_batch(sw_batch b) {
    if (!b) return SW_OK;
    if (b->exec.st) (void)hipStreamSynchronize(b->exec.st);
    delete b;
    return SW_OK;
}

const char* sw_batch_last_error(sw_batch b) { return b ? b->err.c_str() : "null batch"; }

sw_status sw_solve_batch(sw_batch b, const sw_stream* streams, int32_t n, const float* const* depths,
                         int32_t on_device, sw_frame_stats* stats, sw_status* status) {
    if (!b) return SW_EINVAL;
    if (!streams || !depths) return fail(b->err, SW_EINVAL, "streams and depths must not be NULL");
    if (n < 1 || n > kMaxBatch) return fail(b->err, SW_EINVAL, "batch size must be in [1, 64]");
    if (on_device != 0 && on_device != 1) return fail(b->err, SW_EINVAL, "on_device must be 0 or 1");
    std::vector<sw_stream> ss(streams, streams + n);
    for (int i = 0; i < n; ++i) {
        if (!ss[i] || !depths[i]) return fail(b->err, SW_EINVAL, "NULL stream or depth in the batch");
        if (!ss[i]->graph_set)
            return fail(b->err, SW_ESTATE, "every stream needs surfels and a node graph before solving");
        if (ss[i]->server) return fail(b->err, SW_ESTATE, "a stream in the batch is attached to a server");
        for (int j = 0; j < i; ++j)
            if (ss[j] == ss[i]) return fail(b->err, SW_EINVAL, "a stream appears twice in the batch");
    }
    std::vector<sw_status> st(n, SW_OK);
    const sw_status rc = guarded(b->err, [&]() -> sw_status {
        return solve_frames(b->exec, ss, depths, on_device, (b->flags & SW_BATCH_TIMING) != 0, stats, st.data());
    });
    if (status)
        for (int i = 0; i < n; ++i) status[i] = rc == SW_OK || rc == SW_ENUMERIC ? st[i] : rc;
    if (rc == SW_ENUMERIC) b->err = "one or more streams failed numerically; their transforms were restored";
    return rc;
}

sw_status sw_profile_stage(sw_batch b, const sw_stream* streams, int32_t n, int32_t stage, int32_t pcg_it,
                           int32_t reps, float* us_per_launch) {
    if (!b) return SW_EINVAL;
    if (!streams || !us_per_launch) return fail(b->err, SW_EINVAL, "streams and output must not be NULL");
    if (n < 1 || n > kMaxBatch) return fail(b->err, SW_EINVAL, "batch size must be in [1, 64]");
    if (reps < 1 || reps > 100000) return fail(b->err, SW_EINVAL, "reps must be in [1, 100000]");
    const bool replayable = stage == kStWarp || stage == kStCorr || stage == kStAsmFold ||
                            stage == kStPcgInit || stage == kStSpmv || stage == kStUpdate || stage == kStPcgStep;
    if (!replayable) return fail(b->err, SW_EINVAL, "stage cannot be replayed (it reads input or moves nodes)");
    std::vector<sw_stream> ss(streams, streams + n);
    for (int i = 0; i < n; ++i) {
        if (!ss[i]) return fail(b->err, SW_EINVAL, "NULL stream in the batch");
        if (!ss[i]->graph_set) return fail(b->err, SW_ESTATE, "every stream needs a node graph");
        if (ss[i]->server) return fail(b->err, SW_ESTATE, "a stream in the batch is attached to a server");
        if (pcg_it < 0 || pcg_it >= std::max(1, ss[i]->h.pcg_iters))
            return fail(b->err, SW_EINVAL, "pcg_it out of range");
        if (stage == kStPcgStep && pcg_it < 1) return fail(b->err, SW_EINVAL, "a fused step needs pcg_it >= 1");
    }
    return guarded(b->err, [&]() -> sw_status {
        std::vector<int> its(n, 0), ev;
        b->exec.bucket = shape_bucket(ss);
        run_stage(b->exec, stage, ss, its, pcg_it, nullptr, false, ev);   // warm
        hipEvent_t e0 = b->exec.event(0), e1 = b->exec.event(1);
        SWGN_HIP(hipEventRecord(e0, b->exec.st));
        for (int r = 0; r < reps; ++r) run_stage(b->exec, stage, ss, its, pcg_it, nullptr, false, ev);
        SWGN_HIP(hipEventRecord(e1, b->exec.st));
        SWGN_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        SWGN_HIP(hipEventElapsedTime(&ms, e0, e1));
        *us_per_launch = 1000.f * ms / (float)reps;
        return SW_OK;
    });
}

sw_status sw_batch_autotune(sw_batch b, const sw_stream* streams, int32_t n, int32_t reps, int32_t* variants) {
    if (!b) return SW_EINVAL;
    if (!streams) return fail(b->err, SW_EINVAL, "streams must not be NULL");
    if (n < 1 || n > kMaxBatch) return fail(b->err, SW_EINVAL, "batch size must be in [1, 64]");
    if (reps < 1 || reps > 10000) return fail(b->err, SW_EINVAL, "reps must be in [1, 10000]");
    std::vector<sw_stream> ss(streams, streams + n);
    for (int i = 0; i < n; ++i) {
        if (!ss[i]) return fail(b->err, SW_EINVAL, "NULL stream in the batch");
        if (!ss[i]->graph_set) return fail(b->err, SW_ESTATE, "every stream needs a node graph");
        if (ss[i]->server) return fail(b->err, SW_ESTATE, "a stream in the batch is attached to a server");
    }
    return guarded(b->err, [&]() -> sw_status {
        Executor& ex = b->exec;
        const uint64_t key = shape_bucket(ss);
        std::vector<int> choice(kNumStages, 0);
        int pmax = 0;
        for (sw_stream s : ss) pmax = std::max(pmax, s->h.pcg_iters);
        // (the start of PCG runs inside the fold, so its own launch is not tuned)
        const int stages[] = {kStWarp, kStCorr, kStAsmFold, kStSpmv, kStUpdate, kStPcgStep};
        float best_ms[kNumStages] = {0.f};
        std::vector<int> its(n, 0), ev;
        for (int stage : stages) {
            const bool has_wide = stage == kStSpmv || stage == kStUpdate;
            if (stage == kStPcgStep && pmax < 2) continue;
            float best = 0.f;
            bool first = true;
            for (int variant = 0; variant < (has_wide ? 4 : 2); ++variant) {
                // time `reps` back-to-back launches of the stage in this variant
                std::vector<int> trial = choice;
                trial[stage] = variant;
                ex.tuned[key] = trial;
                ex.bucket = key;
                const int pit = (has_wide || stage == kStPcgStep) ? 1 : 0;
                run_stage(ex, stage, ss, its, pit, nullptr, false, ev);
                hipEvent_t e0 = ex.event(0), e1 = ex.event(1);
                SWGN_HIP(hipEventRecord(e0, ex.st));
                for (int r = 0; r < reps; ++r) run_stage(ex, stage, ss, its, pit, nullptr, false, ev);
                SWGN_HIP(hipEventRecord(e1, ex.st));
                SWGN_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                SWGN_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (first || ms < best) {
                    best = ms;
                    choice[stage] = variant;
                    first = false;
                }
            }
            best_ms[stage] = best;
        }
        // one fused step per PCG iteration, or a product and a finish launch
        if (pmax >= 2 && best_ms[kStPcgStep] < best_ms[kStSpmv] + best_ms[kStUpdate]) choice[kStSpmv] |= kVarFused;
        ex.tuned[key] = choice;
        ex.tune_epoch += 1;
        if (variants)
            for (int k = 0; k < 12; ++k) variants[k] = choice[k];
        return SW_OK;
    });
}

}  // extern "C"
