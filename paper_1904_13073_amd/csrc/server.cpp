// Serving loop: frames of many streams arrive at any time and are solved with
// continuous batching.
//
// The server owns one HIP stream, one device slab for frame workspaces and a
// worker thread. A submitted frame waits in FIFO order until (a) its stream
// has no other frame in flight, (b) a batch slot is free and (c) its
// stream's workspace fits in a free range of the slab (admission by HBM
// footprint). The worker then runs steps: one step is one Gauss-Newton
// iteration of every frame in flight, all in the same launches (frames
// admitted in this step first get their depth preprocessing), so a frame that
// arrives while others are on the GPU joins them at the next iteration
// boundary instead of waiting for their whole solve. A frame that completes
// its last iteration has its statistics collected, its workspace returned
// and its ticket marked done. Each workgroup computes from its own stream's
// data only, so a frame's result is the same alone or in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime_internal.h"
#include "swgn.h"
#include "swgn_frame.h"

using namespace swgn;
using namespace swgn::rt;

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator of 256-byte-aligned ranges of the slab.
class RangeAlloc {
public:
    void reset(size_t bytes) {
        free_.clear();
        if (bytes) free_[0] = bytes;
        used_ = 0;
    }
    bool take(size_t bytes, size_t& off) {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const size_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }

private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

struct Ticket {
    uint64_t id = 0;
    sw_stream s = nullptr;
    const float* depth = nullptr;   // device image, or the staging copy of a host one
    int32_t on_device = 0;
    std::vector<float> host_copy;   // host image, copied at submission
    double t_submit = 0, t_admit = 0, t_done = 0;
    bool done = false;
    sw_status status = SW_OK;
    sw_frame_stats stats{};
};

struct Active {
    Ticket* t;
    int it;          // next Gauss-Newton iteration
    size_t off, bytes;
};

}  // namespace

struct sw_server_s {
    Executor exec;
    std::string err;
    int max_batch = kMaxBatch;
    char* slab = nullptr;
    size_t slab_bytes = 0;
    Arena slab_mem;
    RangeAlloc ranges;
    int device = 0;
    Clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    std::string worker_err;

    std::deque<Ticket*> pending;
    std::vector<Active> active;
    std::unordered_map<uint64_t, std::unique_ptr<Ticket>> tickets;
    std::unordered_map<sw_stream, int> attached;   // stream -> frames submitted and not done
    uint64_t next_id = 1;

    // counters
    int64_t steps = 0, frames_done = 0;
    int max_in_flight = 0;
    size_t peak_bytes = 0;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void run();
};

namespace {

// Points the stream's descriptor at a workspace range of the slab and queues
// the descriptor copy on the server's stream (ordered before the kernels).
void bind_workspace(sw_server_s* sv, sw_stream s, size_t off) {
    carve_workspace(s->h, sv->slab + off);
    *s->h_pinned = s->h;
    SWGN_HIP(hipMemcpyAsync(s->d_desc, s->h_pinned, sizeof(FrameDesc), hipMemcpyHostToDevice, sv->exec.st));
}

}  // namespace

void sw_server_s::run() {
    (void)hipSetDevice(device);
    std::vector<sw_stream> ss;
    std::vector<int> its;
    std::vector<char> captured;
    std::vector<int> ev;
    for (;;) {
        std::vector<Ticket*> admitted;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !pending.empty() || !active.empty(); });
            if (stop && active.empty() && pending.empty()) return;
            // admission in arrival order; a stream's frames stay in order
            for (auto it = pending.begin(); it != pending.end() && (int)active.size() < max_batch;) {
                Ticket* t = *it;
                bool busy = false;
                for (const Active& a : active) busy |= (a.t->s == t->s);
                size_t off = 0;
                const size_t bytes = t->s->ws_bytes;
                if (busy || !ranges.take(bytes, off)) {
                    ++it;
                    continue;
                }
                t->t_admit = now();
                active.push_back(Active{t, 0, off, bytes});
                admitted.push_back(t);
                it = pending.erase(it);
            }
            max_in_flight = std::max(max_in_flight, (int)active.size());
            peak_bytes = std::max(peak_bytes, ranges.used());
            if (active.empty()) continue;   // nothing fits yet: wait for more work
        }
        std::vector<Ticket*> finished;
        std::string step_err;
        sw_status rc = guarded(step_err, [&]() -> sw_status {
            // newly admitted frames: workspace, depth in, preprocessing
            std::vector<sw_stream> fresh;
            std::vector<const float*> fresh_depth;
            for (Ticket* t : admitted) {
                size_t off = 0;
                for (const Active& a : active)
                    if (a.t == t) off = a.off;
                bind_workspace(this, t->s, off);
                fresh.push_back(t->s);
                fresh_depth.push_back(t->depth);
            }
            ev.clear();
            if (!fresh.empty()) {
                // device images are read in place; host images (copied at submission) go to the workspace
                std::vector<sw_stream> dev_s, host_s;
                std::vector<const float*> dev_d, host_d;
                for (size_t i = 0; i < admitted.size(); ++i) {
                    if (admitted[i]->on_device) { dev_s.push_back(fresh[i]); dev_d.push_back(fresh_depth[i]); }
                    else { host_s.push_back(fresh[i]); host_d.push_back(fresh_depth[i]); }
                }
                if (!dev_s.empty()) enqueue_depth(exec, dev_s, dev_d.data(), 1, false, ev);
                if (!host_s.empty()) enqueue_depth(exec, host_s, host_d.data(), 0, false, ev);
                enqueue_rigid(exec, fresh, false, ev);
            }
            // one Gauss-Newton iteration of every frame in flight
            ss.clear();
            its.clear();
            for (const Active& a : active) {
                ss.push_back(a.t->s);
                its.push_back(a.it < a.t->s->cfg.gn_iters ? a.it : -1);
            }
            captured.assign(ss.size(), 0);
            enqueue_iteration(exec, ss, its, false, ev, captured);
            for (size_t i = 0; i < active.size(); ++i) {
                if (captured[i]) active[i].t->s->captured = true;
                active[i].it += 1;
            }
            // frames done with their iterations
            std::vector<sw_stream> fs;
            for (const Active& a : active)
                if (a.it >= a.t->s->cfg.gn_iters) {
                    finished.push_back(a.t);
                    fs.push_back(a.t->s);
                }
            if (!fs.empty()) {
                std::vector<sw_frame_stats> st(fs.size());
                std::vector<sw_status> status(fs.size());
                collect_frames(exec, fs, nullptr, st.data(), status.data());
                for (size_t i = 0; i < fs.size(); ++i) {
                    finished[i]->stats = st[i];
                    finished[i]->status = status[i];
                }
            } else {
                SWGN_HIP(hipStreamSynchronize(exec.st));
            }
            return SW_OK;
        });
        std::lock_guard<std::mutex> lk(mu);
        ++steps;
        if (rc != SW_OK) {
            worker_err = step_err;
            // a runtime failure ends every frame in flight with that status
            for (Active& a : active) {
                a.t->status = rc;
                a.t->done = true;
                a.t->t_done = now();
                ranges.give(a.off, a.bytes);
                attached[a.t->s] -= 1;
                ++frames_done;
            }
            active.clear();
            cv_done.notify_all();
            continue;
        }
        const double t = now();
        for (Ticket* f : finished) {
            for (size_t i = 0; i < active.size(); ++i) {
                if (active[i].t != f) continue;
                ranges.give(active[i].off, active[i].bytes);
                active.erase(active.begin() + (long)i);
                break;
            }
            f->done = true;
            f->t_done = t;
            f->host_copy.clear();
            f->host_copy.shrink_to_fit();
            attached[f->s] -= 1;
            ++frames_done;
        }
        if (!finished.empty()) cv_done.notify_all();
    }
}

namespace swgn {
namespace rt {

// Blocks until the stream has no submitted frame that is not done.
void server_quiesce(sw_server sv, sw_stream s) {
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [&] {
        auto it = sv->attached.find(s);
        return it == sv->attached.end() || it->second == 0;
    });
}

// Drops the stream from the server once its frames are done (the stream is
// being destroyed).
void server_forget(sw_server sv, sw_stream s) {
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [&] {
        auto it = sv->attached.find(s);
        return it == sv->attached.end() || it->second == 0;
    });
    sv->attached.erase(s);
    s->server = nullptr;
}

}  // namespace rt
}  // namespace swgn

extern "C" {

void sw_server_config_default(sw_server_config* c) {
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->max_batch = 32;
    c->workspace_bytes = (int64_t)4 << 30;
}

sw_status sw_create_server(const sw_server_config* cfg, void* hip_stream, sw_server* out) {
    if (!out) return SW_EINVAL;
    *out = nullptr;
    if (!cfg || cfg->max_batch < 1 || cfg->max_batch > kMaxBatch || cfg->workspace_bytes < 4096)
        return SW_EINVAL;
    sw_server_s* sv = new (std::nothrow) sw_server_s();
    if (!sv) return SW_ENOMEM;
    const sw_status rc = guarded(sv->err, [&]() -> sw_status {
        SWGN_HIP(hipGetDevice(&sv->device));
        sv->exec.init(hip_stream);
        sv->max_batch = cfg->max_batch;
        sv->slab_bytes = (size_t)cfg->workspace_bytes & ~size_t(255);
        sv->slab = static_cast<char*>(sv->slab_mem.raw(sv->slab_bytes));
        sv->ranges.reset(sv->slab_bytes);
        sv->t0 = Clock::now();
        sv->worker = std::thread([sv] { sv->run(); });
        return SW_OK;
    });
    if (rc != SW_OK) {
        delete sv;
        return rc;
    }
    *out = sv;
    return SW_OK;
}

const char* sw_server_last_error(sw_server sv) { return sv ? sv->err.c_str() : "null server"; }

sw_status sw_server_attach(sw_server sv, sw_stream s) {
    if (!sv || !s) return SW_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (!s->graph_set) return fail(sv->err, SW_ESTATE, "the stream needs surfels and a node graph");
    if (s->server) return fail(sv->err, SW_ESTATE, "the stream is already attached to a server");
    if (s->ws_bytes > sv->slab_bytes)
        return fail(sv->err, SW_EINVAL, "the stream's frame workspace exceeds the server's workspace budget");
    return guarded(sv->err, [&]() -> sw_status {
        // the stream's own workspace goes back to the device; frames use the slab
        SWGN_HIP(hipStreamSynchronize(s->exec.st));
        s->ws_mem.release();
        s->server = sv;
        sv->attached[s] = 0;
        return SW_OK;
    });
}

sw_status sw_server_detach(sw_server sv, sw_stream s) {
    if (!sv || !s) return SW_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->attached.find(s);
    if (it == sv->attached.end()) return fail(sv->err, SW_EINVAL, "the stream is not attached to this server");
    sv->cv_done.wait(lk, [&] { return sv->attached[s] == 0; });
    sv->attached.erase(s);
    s->server = nullptr;
    return guarded(sv->err, [&]() -> sw_status {
        char* ws = static_cast<char*>(s->ws_mem.raw(s->ws_bytes));
        carve_workspace(s->h, ws);
        *s->h_pinned = s->h;
        SWGN_HIP(hipMemcpyAsync(s->d_desc, s->h_pinned, sizeof(FrameDesc), hipMemcpyHostToDevice, s->exec.st));
        SWGN_HIP(hipStreamSynchronize(s->exec.st));
        return SW_OK;
    });
}

sw_status sw_server_submit(sw_server sv, sw_stream s, const float* depth, int32_t on_device, uint64_t* ticket) {
    if (!sv || !s || !depth || !ticket) return SW_EINVAL;
    if (on_device != 0 && on_device != 1) return fail(sv->err, SW_EINVAL, "on_device must be 0 or 1");
    std::unique_ptr<Ticket> t(new (std::nothrow) Ticket());
    if (!t) return SW_ENOMEM;
    t->s = s;
    t->on_device = on_device;
    if (on_device) {
        t->depth = depth;
    } else {
        try {
            t->host_copy.assign(depth, depth + (size_t)s->h.npx);
        } catch (const std::bad_alloc&) {
            return fail(sv->err, SW_ENOMEM, "host allocation failed");
        }
        t->depth = t->host_copy.data();
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    if (s->server != sv) return fail(sv->err, SW_ESTATE, "the stream is not attached to this server");
    if (!sv->worker_err.empty()) return fail(sv->err, SW_EHIP, sv->worker_err);
    t->id = sv->next_id++;
    t->t_submit = sv->now();
    *ticket = t->id;
    sv->attached[s] += 1;
    sv->pending.push_back(t.get());
    sv->tickets[t->id] = std::move(t);
    sv->cv_work.notify_one();
    return SW_OK;
}

sw_status sw_server_poll(sw_server sv, uint64_t ticket, int32_t wait_ms, sw_frame_stats* stats,
                         sw_ticket_info* info) {
    if (!sv) return SW_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return fail(sv->err, SW_EINVAL, "unknown or already collected ticket");
    Ticket* t = it->second.get();
    if (!t->done && wait_ms != 0) {
        auto ready = [&] { return t->done; };
        if (wait_ms < 0) sv->cv_done.wait(lk, ready);
        else sv->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), ready);
    }
    if (!t->done) return SW_EPENDING;
    if (stats) *stats = t->stats;
    if (info) {
        info->status = t->status;
        info->t_submit = t->t_submit;
        info->t_admit = t->t_admit;
        info->t_done = t->t_done;
    }
    sv->tickets.erase(it);
    return SW_OK;
}

sw_status sw_server_counters(sw_server sv, sw_server_info* out) {
    if (!sv || !out) return SW_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    out->steps = sv->steps;
    out->frames_done = sv->frames_done;
    out->max_in_flight = sv->max_in_flight;
    out->pending = (int32_t)sv->pending.size();
    out->in_flight = (int32_t)sv->active.size();
    out->workspace_bytes = (int64_t)sv->slab_bytes;
    out->workspace_peak = (int64_t)sv->peak_bytes;
    return SW_OK;
}

sw_status sw_destroy_server(sw_server sv) {
    if (!sv) return SW_OK;
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->cv_done.wait(lk, [&] { return sv->pending.empty() && sv->active.empty(); });
        sv->stop = true;
        sv->cv_work.notify_all();
    }
    if (sv->worker.joinable()) sv->worker.join();
    // streams still attached get their own workspace back
    std::vector<sw_stream> left;
    for (auto& kv : sv->attached) left.push_back(kv.first);
    for (sw_stream s : left) {
        s->server = nullptr;
        (void)guarded(s->err, [&]() -> sw_status {
            char* ws = static_cast<char*>(s->ws_mem.raw(s->ws_bytes));
            carve_workspace(s->h, ws);
            *s->h_pinned = s->h;
            SWGN_HIP(hipMemcpyAsync(s->d_desc, s->h_pinned, sizeof(FrameDesc), hipMemcpyHostToDevice, s->exec.st));
            SWGN_HIP(hipStreamSynchronize(s->exec.st));
            return SW_OK;
        });
    }
    if (sv->exec.st) (void)hipStreamSynchronize(sv->exec.st);
    delete sv;
    return SW_OK;
}

}  // extern "C"
