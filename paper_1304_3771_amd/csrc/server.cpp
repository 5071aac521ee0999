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
//     become completions and their guest threads become ready again;
//   - a guest thread may also queue a map batch (devirt_map_pages: the
//     backend mapping pages into the process, section 4.2) between its
//     copies.  It runs in the thread's order, once every batch already on the
//     GPU has finished (a table write must not race a walk), and nothing is
//     admitted while it waits or runs.
// Page tables stay resident in the context throughout.
#include <errno.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
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

// A map batch queued as an operation: its maps and results in pinned,
// device-visible memory, the pool, and the caller's result array.  A guest
// table batch (devirt_map_pages) or an EPT batch of VM `vm`
// (devirt_ept_map_pages; its records have the same layout).
struct MapJob {
    uint32_t n = 0;
    bool ept = false;
    uint32_t vm = 0;
    devirt_map *maps = nullptr;
    devirt_result *res = nullptr;
    uint64_t *used = nullptr;
    std::vector<uint64_t> pool;
    devirt_result *res_host = nullptr;
    ~MapJob() {
        hipHostFree(maps);
        hipHostFree(res);
        hipHostFree(used);
    }
};

// An operation: plain data (64 bytes), copied without allocation on its way
// from the inbox through its guest thread's FIFO into a launch.
constexpr uint32_t kNoOp = ~0u;
struct Op {
    uint64_t ticket;
    devirt_request r;  // a map batch: asid and tag only (len 0)
    uint64_t t_submit;
    uint32_t th;       // index of its guest thread (set by the loop)
    uint32_t next;     // the next operation of its guest thread (op pool index)
    MapJob *map;       // non-null: a map batch, owned by the operation until it runs
};

// A guest thread (asid, tag): its waiting operations, a FIFO linked through
// the op pool, and whether one of its operations is in flight.
struct GThread {
    uint32_t head = kNoOp, tail = kNoOp;
    bool busy = false;
    bool empty() const { return head == kNoOp; }
};

// A launch slot: its own stream and workspace, and pinned host buffers that
// the kernels read descriptors from and write results to directly (no
// staging copies on the way in or out).
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    hipEvent_t t_start = nullptr, t_end = nullptr;  // DEVIRT_SERVE_DEVICE_TIMES: the batch's window
    devirt_server *srv = nullptr;  // for the completion host function
    uint32_t idx = 0;
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
    uint32_t mode = 0;          // DEVIRT_SERVE_POLL / NOTIFY / BLOCKING
    bool device_times = false;  // DEVIRT_SERVE_DEVICE_TIMES
    hipEvent_t t_ref = nullptr; // device-time origin, recorded at start
    std::thread th;
    std::atomic<bool> stop{false};
    std::atomic<int> err{0};
    std::string err_msg;

    std::mutex mu;  // guards inbox and done
    std::condition_variable wake;  // submit or a finished batch -> sleeping loop
    std::atomic<uint32_t> done_bits{0};  // DEVIRT_SERVE_NOTIFY: slots whose batch finished
    std::vector<Op> inbox;                // swapped out whole by the loop
    std::vector<devirt_completion> done;  // completions [done_head, size) not yet polled
    size_t done_head = 0;
    uint64_t next_ticket = 0;
    std::atomic<uint64_t> submitted{0}, completed{0};

    // owned by the loop thread: guest threads by index (one hash lookup per
    // operation, at intake), indices of ready threads
    std::unordered_map<uint64_t, uint32_t> tindex;
    std::vector<GThread> threads;
    std::vector<Op> ops;               // op pool: queued operations of every guest thread
    std::vector<uint32_t> free_ops;    // unused op pool entries
    std::deque<uint32_t> ready;
    std::vector<devirt_completion> outbuf;
    uint64_t inflight_ops = 0, inflight_bytes = 0;
    std::vector<Slot> slots;
    uint64_t launches = 0;
    // time accounting (written by the loop thread, read by any)
    std::atomic<uint64_t> st_loops{0}, st_launches{0}, st_ops{0}, st_direct{0};
    std::atomic<uint64_t> ns_inbox{0}, ns_complete{0}, ns_admit{0}, ns_launch{0};
};

// The op pool (loop thread only): a guest thread's FIFO of queued operations.
static void fifo_push(devirt_server *s, GThread &g, const Op &op) {
    uint32_t i;
    if (!s->free_ops.empty()) {
        i = s->free_ops.back();
        s->free_ops.pop_back();
    } else {
        i = (uint32_t)s->ops.size();
        s->ops.emplace_back();
    }
    Op &o = s->ops[i];
    o = op;
    o.next = kNoOp;
    if (g.tail == kNoOp)
        g.head = i;
    else
        s->ops[g.tail].next = i;
    g.tail = i;
}
static const Op &fifo_front(const devirt_server *s, const GThread &g) { return s->ops[g.head]; }
static void fifo_pop(devirt_server *s, GThread &g) {
    const uint32_t i = g.head;
    g.head = s->ops[i].next;
    if (g.head == kNoOp) g.tail = kNoOp;
    s->free_ops.push_back(i);
}

static thread_local bool tl_server_thread = false;
bool dv_in_server_thread() { return tl_server_thread; }

static uint64_t thread_key(const devirt_request &r) { return ((uint64_t)r.asid << 32) | r.tag; }

// Host function run by the HIP runtime once a batch has finished
// (DEVIRT_SERVE_NOTIFY).  It makes no HIP call.
static void on_batch_done(void *arg) {
    Slot *sl = (Slot *)arg;
    devirt_server *s = sl->srv;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->done_bits.fetch_or(1u << sl->idx, std::memory_order_release);
    }
    s->wake.notify_one();
}

// A launch this small (operations, bytes, largest operation) may run as one
// kernel whose translating wavefronts also copy: fewer launches, less latency.
// Larger operations go through the copy queue, where every wavefront helps.
static constexpr uint32_t kDirectOps = 64;
static constexpr uint64_t kDirectBytes = 256 << 10, kDirectMaxOp = 64 << 10;

static int launch_slot(devirt_server *s, Slot &sl) {
    const uint32_t n = (uint32_t)sl.ops.size();
    uint64_t total = 0, largest = 0;
    for (uint32_t i = 0; i < n; ++i) {
        sl.h_reqs[i] = sl.ops[i].r;
        total += sl.ops[i].r.len;
        largest = std::max<uint64_t>(largest, sl.ops[i].r.len);
    }
    const bool direct = n <= kDirectOps && total <= kDirectBytes && largest <= kDirectMaxOp;
    const uint64_t t0 = now_ns();
    if (s->device_times && hipEventRecord(sl.t_start, sl.stream) != hipSuccess)
        return dv_fail(-EIO, "server: event record failed");
    int rc = dv_submit(s->ctx, sl.h_reqs, n, nullptr, 0, sl.h_res, nullptr, nullptr, nullptr, sl.stream, false,
                       direct);
    if (rc) return rc;
    if (s->device_times && hipEventRecord(sl.t_end, sl.stream) != hipSuccess)
        return dv_fail(-EIO, "server: event record failed");
    if (direct) s->st_direct++;
    if (hipEventRecord(sl.ev, sl.stream) != hipSuccess) return dv_fail(-EIO, "server: event record failed");
    if (s->mode == DEVIRT_SERVE_NOTIFY &&
        hipLaunchHostFunc(sl.stream, on_batch_done, &sl) != hipSuccess)
        return dv_fail(-EIO, "server: cannot enqueue the completion function");
    if (s->mode == DEVIRT_SERVE_BLOCKING && hipStreamSynchronize(sl.stream) != hipSuccess)
        return dv_fail(-EIO, "server: batch failed");
    s->ns_launch += now_ns() - t0;
    sl.busy = true;
    s->launches++;
    s->st_launches++;
    return 0;
}

// Runs the map batch at the head of the ready queue (nothing is on the GPU):
// devirt_map_pages or devirt_ept_map_pages on the first slot's stream, waited
// for; its completion summarizes the maps (bytes_done = 4096 per map that
// succeeded; code, level and fault_gva of the first that failed) and the
// caller's array receives every map's result.
static int run_map(devirt_server *s) {
    const uint32_t ti = s->ready.front();
    s->ready.pop_front();
    GThread &g = s->threads[ti];
    const Op op = fifo_front(s, g);
    fifo_pop(s, g);
    const uint64_t t_admit = now_ns();
    std::unique_ptr<MapJob> owned(op.map);
    MapJob &j = *owned;
    hipStream_t st = s->slots[0].stream;
    const uint64_t *pool = j.pool.empty() ? nullptr : j.pool.data();
    int rc = j.ept ? devirt_ept_map_pages(s->ctx, j.vm, (const devirt_ept_map *)j.maps, j.n, pool, j.pool.size(),
                                          j.res, j.used, st)
                   : devirt_map_pages(s->ctx, op.r.asid, j.maps, j.n, pool, j.pool.size(), j.res, j.used, st);
    if (rc) return rc;
    if (hipStreamSynchronize(st) != hipSuccess) return dv_fail(-EIO, "server: map batch failed");
    devirt_completion c;
    memset(&c, 0, sizeof c);
    c.ticket = op.ticket;
    bool failed = false;
    for (uint32_t i = 0; i < j.n; ++i) {
        if (j.res[i].code == DEVIRT_OK) {
            c.res.bytes_done += 4096;
        } else if (!failed) {
            failed = true;
            c.res.code = j.res[i].code;
            c.res.level = j.res[i].level;
            c.res.fault_gva = j.res[i].fault_gva;
        }
    }
    if (j.n) memcpy(j.res_host, j.res, (size_t)j.n * sizeof(devirt_result));
    c.t_submit_ns = op.t_submit;
    c.t_admit_ns = t_admit;
    c.t_done_ns = now_ns();
    if (!g.empty()) s->ready.push_back(ti);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->done.push_back(c);
    }
    s->completed += 1;
    s->st_ops += 1;
    return 0;
}

static void server_loop(devirt_server *s) {
    tl_server_thread = true;
    hipSetDevice(s->ctx->device);
    std::vector<Op> in;
    in.reserve(1 << 12);
    const uint32_t max_batch = s->cfg.max_batch ? s->cfg.max_batch : s->cfg.max_inflight;
    uint64_t taken = 0;  // operations moved out of the inbox so far
    for (;;) {
        bool progress = false;
        const uint64_t t_a = now_ns();
        s->st_loops++;
        // the lock is taken only when something was submitted: a loop that
        // spins on the mutex would keep submitters waiting for it
        if (s->submitted.load(std::memory_order_acquire) != taken) {
            std::lock_guard<std::mutex> g(s->mu);
            in.swap(s->inbox);
            taken += in.size();
        }
        for (auto &op : in) {
            auto it = s->tindex.find(thread_key(op.r));
            if (it == s->tindex.end()) {
                it = s->tindex.emplace(thread_key(op.r), (uint32_t)s->threads.size()).first;
                s->threads.emplace_back();
            }
            op.th = it->second;
            GThread &g = s->threads[op.th];
            if (g.empty() && !g.busy) s->ready.push_back(op.th);
            fifo_push(s, g, op);
            progress = true;
        }
        in.clear();
        const uint64_t t_b = now_ns();
        s->ns_inbox += t_b - t_a;
        // completions
        for (auto &sl : s->slots) {
            if (!sl.busy) continue;
            if (s->mode == DEVIRT_SERVE_NOTIFY) {
                const uint32_t bit = 1u << sl.idx;
                if (!(s->done_bits.load(std::memory_order_acquire) & bit)) continue;
                s->done_bits.fetch_and(~bit, std::memory_order_relaxed);
            }
            hipError_t q = hipEventQuery(sl.ev);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                s->err_msg = hipGetErrorString(q);
                s->err = -EIO;
                sl.busy = false;
                continue;
            }
            const uint64_t t = now_ns();
            uint64_t d0 = 0, d1 = 0;
            if (s->device_times) {
                float a = 0, b = 0;
                if (hipEventElapsedTime(&a, s->t_ref, sl.t_start) == hipSuccess &&
                    hipEventElapsedTime(&b, s->t_ref, sl.t_end) == hipSuccess) {
                    d0 = (uint64_t)((double)a * 1e6);
                    d1 = (uint64_t)((double)b * 1e6);
                }
            }
            std::vector<devirt_completion> &out = s->outbuf;
            out.resize(sl.ops.size());
            for (size_t i = 0; i < sl.ops.size(); ++i) {
                const Op &op = sl.ops[i];
                out[i].ticket = op.ticket;
                out[i].res = sl.h_res[i];
                out[i].t_submit_ns = op.t_submit;
                out[i].t_admit_ns = sl.t_admit[i];
                out[i].t_done_ns = t;
                out[i].dev_start_ns = d0;
                out[i].dev_end_ns = d1;
                GThread &g = s->threads[op.th];
                g.busy = false;
                if (!g.empty()) s->ready.push_back(op.th);
                s->inflight_ops--;
                s->inflight_bytes -= op.r.len;
            }
            {
                std::lock_guard<std::mutex> g(s->mu);
                s->done.insert(s->done.end(), out.begin(), out.end());
            }
            s->completed += sl.ops.size();
            s->st_ops += sl.ops.size();
            sl.ops.clear();
            sl.t_admit.clear();
            sl.busy = false;
            progress = true;
        }
        const uint64_t t_c = now_ns();
        s->ns_complete += t_c - t_b;
        // admission into free slots
        const uint64_t launch_before = s->ns_launch.load();
        if (!s->err) {
            for (auto &sl : s->slots) {
                if (sl.busy || s->ready.empty()) continue;
                const uint64_t t = now_ns();
                while (!s->ready.empty() && sl.ops.size() < max_batch && s->inflight_ops < s->cfg.max_inflight) {
                    GThread &g = s->threads[s->ready.front()];
                    const Op &op = fifo_front(s, g);
                    if (op.map) break;  // a map batch runs alone (below)
                    if (s->inflight_ops > 0 && s->inflight_bytes + op.r.len > s->cfg.pool_bytes) break;
                    s->ready.pop_front();
                    sl.ops.push_back(op);
                    sl.t_admit.push_back(t);
                    s->inflight_ops++;
                    s->inflight_bytes += op.r.len;
                    g.busy = true;
                    fifo_pop(s, g);
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
        // a map batch at the head: once nothing is on the GPU
        if (!s->err && !s->ready.empty() && fifo_front(s, s->threads[s->ready.front()]).map) {
            bool idle = true;
            for (auto &sl : s->slots) idle = idle && !sl.busy;
            if (idle) {
                int rc = run_map(s);
                if (rc) {
                    s->err_msg = devirt_last_error();
                    s->err = rc;
                }
                progress = true;
            }
        }
        s->ns_admit += (now_ns() - t_c) - (s->ns_launch.load() - launch_before);
        if (s->stop.load() && s->completed.load() == s->submitted.load()) break;
        if (s->stop.load() && s->err) break;
        if (!progress) {
            bool inflight = false;
            for (auto &sl : s->slots) inflight = inflight || sl.busy;
            if ((inflight && s->mode != DEVIRT_SERVE_NOTIFY) || !s->ready.empty()) {
                // batches on the GPU: poll again soon, without hogging the core
                for (int k = 0; k < 64; ++k) __builtin_ia32_pause();
                std::this_thread::yield();
            } else {
                // nothing to do until something is submitted, a batch reports
                // back (DEVIRT_SERVE_NOTIFY) or stop
                std::unique_lock<std::mutex> g(s->mu);
                s->wake.wait_for(g, std::chrono::milliseconds(1), [&] {
                    return s->stop.load() || s->submitted.load(std::memory_order_acquire) != taken ||
                           s->done_bits.load(std::memory_order_acquire) != 0;
                });
            }
        }
    }
    tl_server_thread = false;
}

static void free_server(devirt_server *s) {
    for (auto &sl : s->slots) {
        if (sl.stream) hipStreamSynchronize(sl.stream);
        hipHostFree(sl.h_reqs);
        hipHostFree(sl.h_res);
        if (sl.ev) hipEventDestroy(sl.ev);
        if (sl.t_start) hipEventDestroy(sl.t_start);
        if (sl.t_end) hipEventDestroy(sl.t_end);
        if (sl.stream) {
            auto it = s->ctx->ws.find(sl.stream);
            if (it != s->ctx->ws.end()) {
                delete it->second;
                s->ctx->ws.erase(it);
            }
            hipStreamDestroy(sl.stream);
        }
    }
    if (s->t_ref) hipEventDestroy(s->t_ref);
    // map batches that never ran (the server stopped on an error)
    for (auto &op : s->inbox) delete op.map;
    for (auto &g : s->threads)
        for (uint32_t i = g.head; i != kNoOp; i = s->ops[i].next) delete s->ops[i].map;
    s->ctx->server = nullptr;
    delete s;
}

extern "C" int devirt_server_start(devirt_ctx *c, const devirt_server_cfg *cfg, devirt_server **out) {
    if (!c || !cfg || !out) return dv_fail(-EINVAL, "NULL argument");
    *out = nullptr;
    if (c->server) return dv_fail(-EBUSY, "a server is already running on this context");
    if (cfg->max_inflight == 0 || cfg->pool_bytes == 0) return dv_fail(-EINVAL, "max_inflight and pool_bytes must be > 0");
    if (cfg->streams < 1 || cfg->streams > 8) return dv_fail(-EINVAL, "streams must be 1..8");
    const uint32_t mode = cfg->flags & ~DEVIRT_SERVE_DEVICE_TIMES;
    if (mode > DEVIRT_SERVE_BLOCKING)
        return dv_fail(-EINVAL, "flags must be one DEVIRT_SERVE_* mode, optionally with DEVIRT_SERVE_DEVICE_TIMES");
    if (hipSetDevice(c->device) != hipSuccess) return dv_fail(-EIO, "hipSetDevice");
    devirt_server *s = new devirt_server();
    s->ctx = c;
    s->cfg = *cfg;
    s->mode = mode;
    s->device_times = (cfg->flags & DEVIRT_SERVE_DEVICE_TIMES) != 0;
    s->inbox.reserve(1 << 12);
    s->ops.reserve(1 << 12);
    c->server = s;
    const uint32_t max_batch = cfg->max_batch ? cfg->max_batch : cfg->max_inflight;
    s->slots.resize(cfg->streams);  // never resized again: host functions keep slot addresses
    for (auto &sl : s->slots) {
        sl.srv = s;
        sl.idx = (uint32_t)(&sl - s->slots.data());
        bool ok = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) == hipSuccess &&
                  hipHostMalloc(&sl.h_reqs, (size_t)max_batch * sizeof(devirt_request),
                                hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
                  hipHostMalloc(&sl.h_res, (size_t)max_batch * sizeof(devirt_result),
                                hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
                  (!s->device_times || (hipEventCreateWithFlags(&sl.t_start, hipEventDisableSystemFence) == hipSuccess &&
                                        hipEventCreateWithFlags(&sl.t_end, hipEventDisableSystemFence) == hipSuccess));
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
    if (s->device_times) {
        // the origin of device times: recorded on a slot stream and waited for
        if (hipEventCreate(&s->t_ref) != hipSuccess || hipEventRecord(s->t_ref, s->slots[0].stream) != hipSuccess ||
            hipEventSynchronize(s->t_ref) != hipSuccess) {
            free_server(s);
            return dv_fail(-EIO, "server: cannot record the device-time origin");
        }
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
    const size_t base = s->inbox.size();
    const uint32_t k = (uint32_t)std::min<size_t>(n, cap - std::min(cap, base));
    s->inbox.resize(base + k);
    Op *o = s->inbox.data() + base;
    for (uint32_t i = 0; i < k; ++i) o[i] = Op{s->next_ticket++, reqs[i], t, 0, kNoOp, nullptr};
    s->submitted += k;
    if (k) s->wake.notify_one();
    if (n_queued) *n_queued = k;
    if (k < n) return dv_fail(-EBUSY, "server inbox full");
    return 0;
}

// Queues a map batch of either kind for guest thread (asid, tag).  The pool
// is checked here, so that a bad pool is the caller's error, not the server's.
// Both kinds of map travel in the same buffer, copied as devirt_map records.
static_assert(sizeof(devirt_ept_map) == sizeof(devirt_map), "one record size for both kinds of map");

static int submit_map_job(devirt_server *s, uint32_t asid, uint32_t tag, bool ept, uint32_t vm, const void *maps_host,
                          uint32_t n, const uint64_t *pool_host, uint32_t n_pool, devirt_result *res_host,
                          uint64_t *ticket) {
    if (!s || (n && (!maps_host || !res_host)) || (n_pool && !pool_host)) return dv_fail(-EINVAL, "NULL argument");
    if (n > dv::kMapMax) return dv_fail(-EINVAL, "at most %llu maps per call", (unsigned long long)dv::kMapMax);
    if (s->err) return dv_fail(s->err, "server failed: %s", s->err_msg.c_str());
    if (((uintptr_t)maps_host & 7) || ((uintptr_t)res_host & 7))
        return dv_fail(-EINVAL, "maps and res must be 8-byte aligned");
    if (ept) {
        int rc = dv_ept_pool_check(s->ctx, vm, pool_host, n_pool);
        if (rc) return rc;
    } else {
        std::vector<uint64_t> hpa;
        int rc = dv_map_pool_check(s->ctx, asid, pool_host, n_pool, hpa);
        if (rc) return rc;
    }
    std::unique_ptr<MapJob> j(new MapJob());
    j->n = n;
    j->ept = ept;
    j->vm = vm;
    const size_t cnt = n ? n : 1;
    if (hipHostMalloc((void **)&j->maps, cnt * sizeof(devirt_map), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostMalloc((void **)&j->res, cnt * sizeof(devirt_result), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostMalloc((void **)&j->used, sizeof(uint64_t), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
        return dv_fail(-ENOMEM, "server: cannot allocate a map batch");
    if (n) memcpy(j->maps, maps_host, (size_t)n * sizeof(devirt_map));
    j->pool.assign(pool_host, pool_host + n_pool);
    j->res_host = res_host;
    devirt_request r;
    memset(&r, 0, sizeof r);
    r.asid = asid;
    r.tag = tag;
    const uint64_t t = now_ns();
    std::lock_guard<std::mutex> g(s->mu);
    if (ticket) *ticket = s->next_ticket;
    s->inbox.push_back(Op{s->next_ticket++, r, t, 0, kNoOp, j.release()});
    s->submitted += 1;
    s->wake.notify_one();
    return 0;
}

extern "C" int devirt_server_submit_map(devirt_server *s, uint32_t asid, uint32_t tag, const devirt_map *maps_host,
                                        uint32_t n, const uint64_t *pool_gpa_host, uint32_t n_pool,
                                        devirt_result *res_host, uint64_t *ticket) {
    return submit_map_job(s, asid, tag, false, 0, maps_host, n, pool_gpa_host, n_pool, res_host, ticket);
}

extern "C" int devirt_server_submit_ept_map(devirt_server *s, uint32_t asid, uint32_t tag, uint32_t vm,
                                            const devirt_ept_map *maps_host, uint32_t n, const uint64_t *pool_host,
                                            uint32_t n_pool, devirt_result *res_host, uint64_t *ticket) {
    return submit_map_job(s, asid, tag, true, vm, maps_host, n, pool_host, n_pool, res_host, ticket);
}

extern "C" int devirt_server_poll(devirt_server *s, devirt_completion *out, uint32_t max, uint32_t *n_out) {
    if (!s || !n_out || (max && !out)) return dv_fail(-EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    const uint32_t k = (uint32_t)std::min<size_t>(max, s->done.size() - s->done_head);
    if (k) memcpy(out, s->done.data() + s->done_head, (size_t)k * sizeof(devirt_completion));
    s->done_head += k;
    if (s->done_head == s->done.size()) {
        s->done.clear();
        s->done_head = 0;
    } else if (s->done_head >= (1u << 16) && 2 * s->done_head >= s->done.size()) {
        s->done.erase(s->done.begin(), s->done.begin() + (ptrdiff_t)s->done_head);  // keep the buffer bounded
        s->done_head = 0;
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
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->wake.notify_one();
    if (s->th.joinable()) s->th.join();
    const int err = s->err;
    std::string msg = s->err_msg;
    free_server(s);
    if (err) return dv_fail(err, "server failed: %s", msg.c_str());
    return 0;
}

extern "C" int devirt_server_get_stats(devirt_server *s, devirt_server_stats *out) {
    if (!s || !out) return dv_fail(-EINVAL, "NULL argument");
    out->loops = s->st_loops.load();
    out->launches = s->st_launches.load();
    out->ops = s->st_ops.load();
    out->ns_inbox = s->ns_inbox.load();
    out->ns_complete = s->ns_complete.load();
    out->ns_admit = s->ns_admit.load();
    out->ns_launch = s->ns_launch.load();
    out->direct_launches = s->st_direct.load();
    return 0;
}
