// Serving loop: continuous batching of forwarded file-operation copies.
//
// The paper's dual-thread design (section 5) lets a guest thread sleep while
// its operation runs on the host and wakes it on completion; at most one
// operation per guest thread is in flight.  Its polling prototype
// (section 7.4) completes operations faster than interrupts.  Here one host
// thread plays the backend for many guests:
//   - operations arrive through devirt_server_submit into an inbox;
//   - each guest thread (asid, tag) has a FIFO; a thread with nothing in
//     flight and a non-empty FIFO is "ready";
//   - whenever a launch slot (stream) is free, ready operations are admitted
//     while descriptor slots and the byte budget allow, written to the slot's
//     pinned buffer and launched as one batch on that slot's stream (the
//     kernels read the descriptors and write results in place), while earlier batches
//     are still running on the other streams (their work overlaps on the
//     GPU);
//   - finished batches are found by polling their events; their results
//     become completions and their guest threads become ready again.
// Page tables stay resident in the context throughout.
#include <errno.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime.h"

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Op {
    uint64_t ticket;
    devirt_request r;
    uint64_t t_submit;
};

// A launch slot: its own stream and workspace, and pinned host buffers that
// the kernels read descriptors from and write results to directly (no
// staging copies on the way in or out).
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    devirt_request *h_reqs = nullptr;  // pinned, device-visible
    devirt_result *h_res = nullptr;    // pinned, device-visible
    std::vector<Op> ops;
    std::vector<uint64_t> t_admit;
    bool busy = false;
};

}  // namespace

struct devirt_server {
    devirt_ctx *ctx = nullptr;
    devirt_server_cfg cfg{};
    std::thread th;
    std::atomic<bool> stop{false};
    std::atomic<int> err{0};
    std::string err_msg;

    std::mutex mu;  // guards inbox and done
    std::deque<Op> inbox;
    std::deque<devirt_completion> done;
    uint64_t next_ticket = 0;
    std::atomic<uint64_t> submitted{0}, completed{0};

    // owned by the loop thread
    std::unordered_map<uint64_t, std::deque<Op>> fifo;
    std::unordered_map<uint64_t, bool> busy;
    std::deque<uint64_t> ready;
    uint64_t inflight_ops = 0, inflight_bytes = 0;
    std::vector<Slot> slots;
    uint64_t launches = 0;
};

static thread_local bool tl_server_thread = false;
bool dv_in_server_thread() { return tl_server_thread; }

static uint64_t thread_key(const devirt_request &r) { return ((uint64_t)r.asid << 32) | r.tag; }

static int launch_slot(devirt_server *s, Slot &sl) {
    const uint32_t n = (uint32_t)sl.ops.size();
    for (uint32_t i = 0; i < n; ++i) sl.h_reqs[i] = sl.ops[i].r;
    int rc = dv_submit(s->ctx, sl.h_reqs, n, nullptr, 0, sl.h_res, nullptr, nullptr, nullptr, sl.stream, false);
    if (rc) return rc;
    if (hipEventRecord(sl.ev, sl.stream) != hipSuccess) return dv_fail(-EIO, "server: event record failed");
    sl.busy = true;
    s->launches++;
    return 0;
}

static void server_loop(devirt_server *s) {
    tl_server_thread = true;
    hipSetDevice(s->ctx->device);
    std::deque<Op> in;
    const uint32_t max_batch = s->cfg.max_batch ? s->cfg.max_batch : s->cfg.max_inflight;
    for (;;) {
        bool progress = false;
        {
            std::lock_guard<std::mutex> g(s->mu);
            in.swap(s->inbox);
        }
        for (auto &op : in) {
            const uint64_t k = thread_key(op.r);
            auto &q = s->fifo[k];
            if (q.empty() && !s->busy[k]) s->ready.push_back(k);
            q.push_back(op);
            progress = true;
        }
        in.clear();
        // completions
        for (auto &sl : s->slots) {
            if (!sl.busy) continue;
            hipError_t q = hipEventQuery(sl.ev);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                s->err_msg = hipGetErrorString(q);
                s->err = -EIO;
                sl.busy = false;
                continue;
            }
            const uint64_t t = now_ns();
            std::vector<devirt_completion> out(sl.ops.size());
            for (size_t i = 0; i < sl.ops.size(); ++i) {
                const Op &op = sl.ops[i];
                out[i].ticket = op.ticket;
                out[i].res = sl.h_res[i];
                out[i].t_submit_ns = op.t_submit;
                out[i].t_admit_ns = sl.t_admit[i];
                out[i].t_done_ns = t;
                const uint64_t k = thread_key(op.r);
                s->busy[k] = false;
                if (!s->fifo[k].empty()) s->ready.push_back(k);
                s->inflight_ops--;
                s->inflight_bytes -= op.r.len;
            }
            {
                std::lock_guard<std::mutex> g(s->mu);
                for (auto &c : out) s->done.push_back(c);
            }
            s->completed += sl.ops.size();
            sl.ops.clear();
            sl.t_admit.clear();
            sl.busy = false;
            progress = true;
        }
        // admission into free slots
        if (!s->err) {
            for (auto &sl : s->slots) {
                if (sl.busy || s->ready.empty()) continue;
                const uint64_t t = now_ns();
                while (!s->ready.empty() && sl.ops.size() < max_batch && s->inflight_ops < s->cfg.max_inflight) {
                    const uint64_t k = s->ready.front();
                    auto &q = s->fifo[k];
                    const Op &op = q.front();
                    if (s->inflight_ops > 0 && s->inflight_bytes + op.r.len > s->cfg.pool_bytes) break;
                    s->ready.pop_front();
                    sl.ops.push_back(op);
                    sl.t_admit.push_back(t);
                    s->inflight_ops++;
                    s->inflight_bytes += op.r.len;
                    s->busy[k] = true;
                    q.pop_front();
                }
                if (sl.ops.empty()) break;
                int rc = launch_slot(s, sl);
                if (rc) {
                    s->err_msg = devirt_last_error();
                    s->err = rc;
                    break;
                }
                progress = true;
            }
        }
        if (s->stop.load() && s->completed.load() == s->submitted.load()) break;
        if (s->stop.load() && s->err) break;
        if (!progress) std::this_thread::yield();
    }
    tl_server_thread = false;
}

static void free_server(devirt_server *s) {
    for (auto &sl : s->slots) {
        if (sl.stream) hipStreamSynchronize(sl.stream);
        hipHostFree(sl.h_reqs);
        hipHostFree(sl.h_res);
        if (sl.ev) hipEventDestroy(sl.ev);
        if (sl.stream) {
            auto it = s->ctx->ws.find(sl.stream);
            if (it != s->ctx->ws.end()) {
                delete it->second;
                s->ctx->ws.erase(it);
            }
            hipStreamDestroy(sl.stream);
        }
    }
    s->ctx->server = nullptr;
    delete s;
}

extern "C" int devirt_server_start(devirt_ctx *c, const devirt_server_cfg *cfg, devirt_server **out) {
    if (!c || !cfg || !out) return dv_fail(-EINVAL, "NULL argument");
    *out = nullptr;
    if (c->server) return dv_fail(-EBUSY, "a server is already running on this context");
    if (cfg->max_inflight == 0 || cfg->pool_bytes == 0) return dv_fail(-EINVAL, "max_inflight and pool_bytes must be > 0");
    if (cfg->streams < 1 || cfg->streams > 8) return dv_fail(-EINVAL, "streams must be 1..8");
    if (cfg->flags != 0) return dv_fail(-EINVAL, "flags must be 0");
    if (hipSetDevice(c->device) != hipSuccess) return dv_fail(-EIO, "hipSetDevice");
    devirt_server *s = new devirt_server();
    s->ctx = c;
    s->cfg = *cfg;
    c->server = s;
    const uint32_t max_batch = cfg->max_batch ? cfg->max_batch : cfg->max_inflight;
    s->slots.resize(cfg->streams);
    for (auto &sl : s->slots) {
        bool ok = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) == hipSuccess &&
                  hipHostMalloc(&sl.h_reqs, (size_t)max_batch * sizeof(devirt_request),
                                hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
                  hipHostMalloc(&sl.h_res, (size_t)max_batch * sizeof(devirt_result),
                                hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess;
        if (!ok) {
            free_server(s);
            return dv_fail(-ENOMEM, "server: cannot allocate launch slots");
        }
        Workspace *w = get_ws(c, sl.stream);
        int rc = ensure_ws(c, w, max_batch, 1, false, 0);
        if (rc) {
            free_server(s);
            return rc;
        }
        sl.ops.reserve(max_batch);
    }
    s->th = std::thread(server_loop, s);
    *out = s;
    return 0;
}

extern "C" int devirt_server_submit(devirt_server *s, const devirt_request *reqs, uint32_t n, uint32_t *n_queued) {
    if (!s || (n && !reqs)) return dv_fail(-EINVAL, "NULL argument");
    if (n_queued) *n_queued = 0;
    if (s->err) return dv_fail(s->err, "server failed: %s", s->err_msg.c_str());
    const uint64_t t = now_ns();
    const size_t cap = 1u << 24;
    std::lock_guard<std::mutex> g(s->mu);
    uint32_t k = 0;
    for (; k < n && s->inbox.size() < cap; ++k) s->inbox.push_back(Op{s->next_ticket++, reqs[k], t});
    s->submitted += k;
    if (n_queued) *n_queued = k;
    if (k < n) return dv_fail(-EBUSY, "server inbox full");
    return 0;
}

extern "C" int devirt_server_poll(devirt_server *s, devirt_completion *out, uint32_t max, uint32_t *n_out) {
    if (!s || !n_out || (max && !out)) return dv_fail(-EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    uint32_t k = 0;
    while (k < max && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *n_out = k;
    if (k == 0 && s->err) return dv_fail(s->err, "server failed: %s", s->err_msg.c_str());
    return 0;
}

extern "C" int devirt_server_drain(devirt_server *s) {
    if (!s) return dv_fail(-EINVAL, "NULL argument");
    while (s->completed.load() < s->submitted.load()) {
        if (s->err) return dv_fail(s->err, "server failed: %s", s->err_msg.c_str());
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    return 0;
}

extern "C" int devirt_server_stop(devirt_server *s) {
    if (!s) return dv_fail(-EINVAL, "NULL argument");
    s->stop = true;
    if (s->th.joinable()) s->th.join();
    const int err = s->err;
    std::string msg = s->err_msg;
    free_server(s);
    if (err) return dv_fail(err, "server failed: %s", msg.c_str());
    return 0;
}
