// Host-side state of a devirt context (shared by the runtime and the server).
#pragma once
#include <stdint.h>

#include <list>
#include <map>
#include <vector>

#include "dv_internal.h"

struct VmHost {
    uint8_t *arena = nullptr;
    uint64_t bytes = 0;
    struct Slot {
        uint64_t gpa = 0, bytes = 0, off = 0;
        bool used = false;
    } slots[64];
    uint64_t *d_index = nullptr;
    dv::DSlot *d_slots = nullptr;
    uint32_t index_len = 0, nsorted = 0, index_complete = 1;
    uint64_t ept_root = ~0ull;  // ~0: translate through the memslots
};

struct GraphEntry {
    uint64_t hash;
    std::vector<uint64_t> key;
    hipGraphExec_t exec;
};

// Per-stream scratch: the copy-segment queue, epoch counters, per-request
// pending counts (completion times), fault-list tile sums, the clock origin
// and the captured graphs that reference them.
struct Workspace {
    hipStream_t stream = nullptr;
    dv::DSeg *segs = nullptr;    // long-segment queue
    uint64_t seg_cap = 0;
    dv::DSeg *shorts = nullptr;  // short-segment queue, same capacity
    uint64_t short_cap = 0;
    dv::DEpochCtr *ctr = nullptr;
    uint64_t ctr_cap = 0;
    uint32_t *pending = nullptr;
    uint64_t pending_cap = 0;
    uint32_t *tiles = nullptr;
    uint64_t tiles_cap = 0;
    uint64_t *t0 = nullptr;
    uint64_t t0_cap = 0;
    uint64_t *spill = nullptr;          // per request slot: groups left to the spill pass
    uint64_t spill_cap = 0;
    uint64_t *large = nullptr;          // per request slot: the epoch's large requests
    uint64_t large_cap = 0;
    std::vector<GraphEntry> graphs;
    hipStream_t side = nullptr;         // translate launches run here, ahead of the copies
    std::vector<hipEvent_t> events;     // per epoch: translate done, copy done; plus the fork
    // devirt_map_pages
    uint64_t *map_buf = nullptr;        // table-key set and lists, page set, scalars, pool
    uint64_t map_cap = 0;
    uint64_t *map_pool_host = nullptr;  // pinned staging of the pool (gpa, hpa)
    uint64_t map_pool_host_cap = 0;
    hipEvent_t map_ev = nullptr;        // the last pool upload
    ~Workspace();
};

struct ProfEv {
    int kind;  // 0 copy, 1 translate
    hipEvent_t a, b;
};

struct devirt_ctx {
    int device = 0;
    int cus = 0;
    uint64_t wall_khz = 100000;
    std::vector<VmHost> vms;
    std::vector<dv::DProc> procs;
    dv::DVm *d_vms = nullptr;
    size_t d_vms_cap = 0;
    dv::DProc *d_procs = nullptr;
    size_t d_procs_cap = 0;
    dv::DFifo *d_fifo = nullptr;  // per process: the per-request path's translation cache
    uint64_t tables_version = 0;
    uint64_t xlat_gen = 1;        // advanced by every change to guest memory or translation setup
    devirt_config cfg;
    uint64_t cfg_version = 0;
    std::map<hipStream_t, Workspace *> ws;
    int profiling = 0;
    devirt_stats stats = {};
    dv::DCounters *d_counters = nullptr;
    std::list<ProfEv> prof;
    void *server = nullptr;  // non-null while a serving loop owns the context
    hipStream_t capture_stream = nullptr;  // private stream batches are captured on
};

struct BatchArgs {
    const devirt_request *reqs = nullptr;
    uint64_t n = 0;
    devirt_result *res = nullptr;
    devirt_fault *faults = nullptr;
    uint64_t *n_faults = nullptr;
    uint64_t *t_done = nullptr;
    std::vector<uint64_t> epochs;
    bool direct = false;  // one translate launch that also copies (small batches)
};

// Device memory of the per-request copy that allocates nothing: one
// request's epoch counters, clock origin and segment queues (cap segments
// each), inside a static device array (static_copy.hip).
struct StaticScratch {
    dv::DEpochCtr *ctr;
    uint64_t *t0;
    dv::DSeg *segs;
    dv::DSeg *shorts;
    uint64_t cap;
};
// Looks the array up on `device` (current) once per process; devirt_open calls it.
int static_scratch_init(int device);
// The per-request copy; with st, into that scratch instead of the stream's workspace.
int plain_copy(devirt_ctx *c, uint32_t asid, uint64_t gva, uint64_t host, uint64_t len, uint32_t dir,
               devirt_result *res, void *stream, const StaticScratch *st);

int dv_fail(int code, const char *fmt, ...);
dv::DView view_of(const devirt_ctx *c);
Workspace *get_ws(devirt_ctx *c, hipStream_t s);
int ensure_ws(devirt_ctx *c, Workspace *w, uint64_t n_req, uint64_t n_epochs, bool need_pending, uint64_t min_segs);
dv::DBatch make_batch(devirt_ctx *c, Workspace *w);
int dv_submit(devirt_ctx *c, const devirt_request *reqs, uint64_t n, const uint64_t *epoch_end, uint32_t n_epochs,
              devirt_result *res, devirt_fault *faults, uint64_t *n_faults, uint64_t *t_done, hipStream_t s,
              bool allow_graph, bool allow_direct = false);
bool dv_in_server_thread();
// Checks a guest-table map batch's pool (devirt_map_pages) and gives each
// frame's arena offset (memslot VMs; zeros for a VM with an EPT).
int dv_map_pool_check(const devirt_ctx *c, uint32_t asid, const uint64_t *pool_gpa, uint64_t n_pool,
                      std::vector<uint64_t> &hpa);
// Checks an EPT map batch's VM and pool (devirt_ept_map_pages).
int dv_ept_pool_check(const devirt_ctx *c, uint32_t vm, const uint64_t *pool_host, uint64_t n_pool);
