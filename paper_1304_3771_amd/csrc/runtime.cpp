// Host runtime of the devirt C ABI: device tables (arenas, memslots with a
// 2 MiB direct index, processes), per-stream workspaces, batch enqueue with
// HIP-graph capture and replay, profiling, configuration and autotuning.
#include <errno.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <string>
#include <vector>

#include "dv_internal.h"
#include "runtime.h"

using namespace dv;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

int dv_fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

extern "C" const char *devirt_last_error(void) { return g_err.c_str(); }

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) return dv_fail(-EIO, "%s: %s", #x, hipGetErrorString(e_));   \
    } while (0)

// ------------------------------------------------------------------ config
static devirt_config default_config() {
    devirt_config c;
    c.group = 64;
    c.seg_chunks = 16;
    c.xlat_wg = 256;
    c.xlat_wgs_per_cu = 1;
    c.copy_wg = 512;
    c.copy_wgs_per_cu = 8;
    c.nontemporal = 0;
    c.inline_bytes = 0;
    c.use_graph = 1;
    c.overlap = 1;
    c.fifo_entries = 0;
    c.large_pages = 0;
    c.spill_side = 1;
    return c;
}

static int check_config(const devirt_config &c) {
    if (c.group < 1 || c.group > 64) return dv_fail(-EINVAL, "group must be 1..64");
    if (c.seg_chunks < 1 || c.seg_chunks > 64) return dv_fail(-EINVAL, "seg_chunks must be 1..64");
    if (c.xlat_wg < 64 || c.xlat_wg > 256 || c.xlat_wg % 64) return dv_fail(-EINVAL, "xlat_wg must be 64..256, x64");
    if (c.copy_wg < 64 || c.copy_wg > 1024 || c.copy_wg % 64) return dv_fail(-EINVAL, "copy_wg must be 64..1024, x64");
    if (c.xlat_wgs_per_cu < 1 || c.xlat_wgs_per_cu > 64) return dv_fail(-EINVAL, "xlat_wgs_per_cu must be 1..64");
    if (c.copy_wgs_per_cu < 1 || c.copy_wgs_per_cu > 64) return dv_fail(-EINVAL, "copy_wgs_per_cu must be 1..64");
    if (c.nontemporal > 1 || c.use_graph > 1) return dv_fail(-EINVAL, "nontemporal/use_graph must be 0 or 1");
    if (c.inline_bytes > 256) return dv_fail(-EINVAL, "inline_bytes must be <= 256");
    if (c.overlap > 1) return dv_fail(-EINVAL, "overlap must be 0 or 1");
    if (c.fifo_entries > kFifoMax) return dv_fail(-EINVAL, "fifo_entries must be <= %u", kFifoMax);
    if (c.large_pages != 0 && c.large_pages < 64) return dv_fail(-EINVAL, "large_pages must be 0 or >= 64");
    if (c.spill_side > 1) return dv_fail(-EINVAL, "spill_side must be 0 or 1");
    return 0;
}

// ------------------------------------------------------------------ context
Workspace::~Workspace() {
    for (auto &g : graphs) hipGraphExecDestroy(g.exec);
    for (auto e : events) hipEventDestroy(e);
    if (side) {
        hipStreamSynchronize(side);
        hipStreamDestroy(side);
    }
    hipFree(segs);
    hipFree(shorts);
    hipFree(ctr);
    hipFree(pending);
    hipFree(tiles);
    hipFree(t0);
    hipFree(spill);
    hipFree(large);
    if (map_ev) {
        hipEventSynchronize(map_ev);
        hipEventDestroy(map_ev);
    }
    hipFree(map_buf);
    hipHostFree(map_pool_host);
}

// While a serving loop runs, only its own thread may drive the context.
static bool server_owns(const devirt_ctx *c) { return c->server != nullptr && !dv_in_server_thread(); }

static int set_dev(devirt_ctx *c) {
    HIPCHK(hipSetDevice(c->device));
    return 0;
}

extern "C" int devirt_open(int hip_device, devirt_ctx **out) {
    if (!out) return dv_fail(-EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (hip_device < 0 || hip_device >= ndev) return dv_fail(-EINVAL, "no HIP device %d (%d present)", hip_device, ndev);
    HIPCHK(hipSetDevice(hip_device));
    int rc = static_scratch_init(hip_device);
    if (rc) return rc;
    devirt_ctx *c = new devirt_ctx();
    c->device = hip_device;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, hip_device) != hipSuccess || v <= 0) {
        delete c;
        return dv_fail(-EIO, "cannot read the CU count");
    }
    c->cus = v;
    v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, hip_device) != hipSuccess || v <= 0) v = 100000;
    c->wall_khz = (uint64_t)v;
    c->cfg = default_config();
    if (hipMalloc(&c->d_counters, sizeof(DCounters)) != hipSuccess) {
        delete c;
        return dv_fail(-ENOMEM, "hipMalloc counters");
    }
    hipMemset(c->d_counters, 0, sizeof(DCounters));
    *out = c;
    return 0;
}

extern "C" int devirt_close(devirt_ctx *c) {
    if (!c) return dv_fail(-EINVAL, "ctx is NULL");
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    for (auto &kv : c->ws) delete kv.second;
    for (auto &vm : c->vms) {
        hipFree(vm.arena);
        hipFree(vm.d_index);
        hipFree(vm.d_slots);
    }
    hipFree(c->d_vms);
    hipFree(c->d_procs);
    hipFree(c->d_fifo);
    hipFree(c->d_counters);
    for (auto &p : c->prof) {
        hipEventDestroy(p.a);
        hipEventDestroy(p.b);
    }
    if (c->capture_stream) hipStreamDestroy(c->capture_stream);
    delete c;
    return 0;
}

// Re-upload the VM table (after a VM or memslot change).  Device must be idle.
static int upload_vms(devirt_ctx *c) {
    std::vector<DVm> h(c->vms.size());
    for (size_t i = 0; i < c->vms.size(); ++i) {
        const VmHost &v = c->vms[i];
        h[i].arena = v.arena;
        h[i].arena_bytes = v.bytes;
        h[i].index = v.d_index;
        h[i].slots = v.d_slots;
        h[i].index_len = v.index_len;
        h[i].nslots = v.nsorted;
        h[i].index_complete = v.index_complete;
        h[i].lds_base = kLdsNone;
        h[i].lds_idx = kLdsNone;
        h[i].ept_root = v.ept_root;
    }
    if (c->vms.size() > c->d_vms_cap) {
        size_t cap = std::max<size_t>(16, c->vms.size() * 2);
        DVm *p = nullptr;
        HIPCHK(hipMalloc(&p, cap * sizeof(DVm)));
        hipFree(c->d_vms);
        c->d_vms = p;
        c->d_vms_cap = cap;
    }
    if (!h.empty()) HIPCHK(hipMemcpy(c->d_vms, h.data(), h.size() * sizeof(DVm), hipMemcpyHostToDevice));
    c->tables_version++;
    c->xlat_gen++;
    return 0;
}

static int upload_procs(devirt_ctx *c) {
    if (c->procs.size() > c->d_procs_cap) {
        size_t cap = std::max<size_t>(64, c->procs.size() * 2);
        DProc *p = nullptr;
        HIPCHK(hipMalloc(&p, cap * sizeof(DProc)));
        DFifo *f = nullptr;
        if (hipMalloc(&f, cap * sizeof(DFifo)) != hipSuccess) {
            hipFree(p);
            return dv_fail(-ENOMEM, "hipMalloc translation caches");
        }
        // new processes start with an empty cache and zero counts (gen 0 never matches)
        HIPCHK(hipMemset(f, 0, cap * sizeof(DFifo)));
        if (c->d_fifo) HIPCHK(hipMemcpy(f, c->d_fifo, c->d_procs_cap * sizeof(DFifo), hipMemcpyDeviceToDevice));
        hipFree(c->d_procs);
        hipFree(c->d_fifo);
        c->d_procs = p;
        c->d_fifo = f;
        c->d_procs_cap = cap;
    }
    if (!c->procs.empty())
        HIPCHK(hipMemcpy(c->d_procs, c->procs.data(), c->procs.size() * sizeof(DProc), hipMemcpyHostToDevice));
    c->tables_version++;
    return 0;
}

extern "C" int devirt_vm_create(devirt_ctx *c, uint64_t arena_bytes, uint32_t *vm) {
    if (!c || !vm) return dv_fail(-EINVAL, "NULL argument");
    if (arena_bytes == 0 || (arena_bytes & 4095)) return dv_fail(-EINVAL, "arena_bytes must be a non-zero multiple of 4096");
    if (server_owns(c)) return dv_fail(-EBUSY, "a serving loop owns this context");
    if (c->vms.size() >= 0xFFFF) return dv_fail(-EINVAL, "too many VMs");
    if (set_dev(c)) return -EIO;
    HIPCHK(hipDeviceSynchronize());
    VmHost v;
    if (hipMalloc(&v.arena, arena_bytes) != hipSuccess) return dv_fail(-ENOMEM, "cannot allocate a %llu-byte arena",
                                                                     (unsigned long long)arena_bytes);
    if (hipMemset(v.arena, 0, arena_bytes) != hipSuccess) {
        hipFree(v.arena);
        return dv_fail(-EIO, "hipMemset arena");
    }
    v.bytes = arena_bytes;
    c->vms.push_back(v);
    int rc = upload_vms(c);
    if (rc) return rc;
    *vm = (uint32_t)(c->vms.size() - 1);
    return 0;
}

extern "C" int devirt_vm_arena(devirt_ctx *c, uint32_t vm, void **dev_ptr, uint64_t *bytes) {
    if (!c) return dv_fail(-EINVAL, "ctx is NULL");
    if (vm >= c->vms.size()) return dv_fail(-ENOENT, "no VM %u", vm);
    if (dev_ptr) *dev_ptr = c->vms[vm].arena;
    if (bytes) *bytes = c->vms[vm].bytes;
    return 0;
}

static int vm_copy(devirt_ctx *c, uint32_t vm, uint64_t off, void *host_or_dev, uint64_t bytes, bool write) {
    if (!c) return dv_fail(-EINVAL, "ctx is NULL");
    if (vm >= c->vms.size()) return dv_fail(-ENOENT, "no VM %u", vm);
    if (bytes == 0) return 0;
    if (server_owns(c)) return dv_fail(-EBUSY, "a serving loop owns this context");
    if (!host_or_dev) return dv_fail(-EINVAL, "NULL buffer");
    const VmHost &v = c->vms[vm];
    if (off > v.bytes || bytes > v.bytes - off) return dv_fail(-EINVAL, "range leaves the arena");
    if (set_dev(c)) return -EIO;
    HIPCHK(hipDeviceSynchronize());
    if (write) {
        HIPCHK(hipMemcpy(v.arena + off, host_or_dev, bytes, hipMemcpyDefault));
        c->xlat_gen++;  // the bytes may be page tables (A/D bits a cached translation relies on)
    } else
        HIPCHK(hipMemcpy(host_or_dev, v.arena + off, bytes, hipMemcpyDefault));
    return 0;
}

extern "C" int devirt_vm_write(devirt_ctx *c, uint32_t vm, uint64_t off, const void *src, uint64_t bytes) {
    return vm_copy(c, vm, off, const_cast<void *>(src), bytes, true);
}
extern "C" int devirt_vm_read(devirt_ctx *c, uint32_t vm, uint64_t off, void *dst, uint64_t bytes) {
    return vm_copy(c, vm, off, dst, bytes, false);
}

// Build the sorted slot list and the 2 MiB direct index of one VM.
static constexpr uint64_t kBlk = 2ull << 20;
static constexpr uint64_t kIndexCap = 1ull << 20;  // blocks: covers 2 TiB of GPA

int build_slot_index(const VmHost &v, std::vector<DSlot> &sorted, std::vector<uint64_t> &index, uint32_t &complete) {
    sorted.clear();
    for (const auto &s : v.slots)
        if (s.used) sorted.push_back(DSlot{s.gpa, s.gpa + s.bytes, s.off});
    std::sort(sorted.begin(), sorted.end(), [](const DSlot &a, const DSlot &b) { return a.gpa < b.gpa; });
    uint64_t max_end = sorted.empty() ? 0 : sorted.back().end;
    uint64_t nblk = (max_end + kBlk - 1) / kBlk;
    complete = 1;
    if (nblk > kIndexCap) {
        nblk = kIndexCap;
        complete = 0;
    }
    index.assign(nblk, 0);
    for (const auto &s : sorted) {
        uint64_t b0 = s.gpa / kBlk, b1 = (s.end - 1) / kBlk;
        for (uint64_t b = b0; b <= b1 && b < nblk; ++b) {
            uint64_t lo = b * kBlk, hi = lo + kBlk;
            if (s.gpa <= lo && s.end >= hi)
                index[b] = (s.arena_off - s.gpa) | 2ull;
            else
                index[b] = 1ull;
        }
    }
    return 0;
}

extern "C" int devirt_memslot_set(devirt_ctx *c, uint32_t vm, uint32_t slot, uint64_t gpa, uint64_t bytes,
                                  uint64_t arena_off) {
    if (!c) return dv_fail(-EINVAL, "ctx is NULL");
    if (vm >= c->vms.size()) return dv_fail(-ENOENT, "no VM %u", vm);
    if (slot >= 64) return dv_fail(-EINVAL, "slot must be 0..63");
    if (server_owns(c)) return dv_fail(-EBUSY, "a serving loop owns this context");
    VmHost &v = c->vms[vm];
    if (bytes != 0) {
        if ((gpa | bytes | arena_off) & 4095) return dv_fail(-EINVAL, "gpa, bytes and arena_off must be 4 KiB aligned");
        if (gpa >= (1ull << 52) || bytes > (1ull << 52) - gpa) return dv_fail(-EINVAL, "slot passes 2^52");
        if (arena_off > v.bytes || bytes > v.bytes - arena_off) return dv_fail(-EINVAL, "slot leaves the arena");
        for (uint32_t i = 0; i < 64; ++i) {
            const auto &o = v.slots[i];
            if (i == slot || !o.used) continue;
            if (gpa < o.gpa + o.bytes && o.gpa < gpa + bytes)
                return dv_fail(-EEXIST, "GPA range overlaps slot %u", i);
        }
    }
    if (set_dev(c)) return -EIO;
    HIPCHK(hipDeviceSynchronize());
    VmHost nv = v;
    nv.slots[slot].used = bytes != 0;
    nv.slots[slot].gpa = gpa;
    nv.slots[slot].bytes = bytes;
    nv.slots[slot].off = arena_off;
    std::vector<DSlot> sorted;
    std::vector<uint64_t> index;
    uint32_t complete = 1;
    build_slot_index(nv, sorted, index, complete);
    DSlot *ds = nullptr;
    uint64_t *di = nullptr;
    if (!sorted.empty()) {
        if (hipMalloc(&ds, sorted.size() * sizeof(DSlot)) != hipSuccess) return dv_fail(-ENOMEM, "hipMalloc slots");
        HIPCHK(hipMemcpy(ds, sorted.data(), sorted.size() * sizeof(DSlot), hipMemcpyHostToDevice));
    }
    if (!index.empty()) {
        if (hipMalloc(&di, index.size() * 8) != hipSuccess) {
            hipFree(ds);
            return dv_fail(-ENOMEM, "hipMalloc slot index");
        }
        HIPCHK(hipMemcpy(di, index.data(), index.size() * 8, hipMemcpyHostToDevice));
    }
    hipFree(v.d_slots);
    hipFree(v.d_index);
    v = nv;
    v.d_slots = ds;
    v.d_index = di;
    v.nsorted = (uint32_t)sorted.size();
    v.index_len = (uint32_t)index.size();
    v.index_complete = complete;
    return upload_vms(c);
}

extern "C" int devirt_vm_set_ept(devirt_ctx *c, uint32_t vm, uint64_t root) {
    if (!c) return dv_fail(-EINVAL, "ctx is NULL");
    if (vm >= c->vms.size()) return dv_fail(-ENOENT, "no VM %u", vm);
    if (server_owns(c)) return dv_fail(-EBUSY, "a serving loop owns this context");
    VmHost &v = c->vms[vm];
    if (root != ~0ull && ((root & 4095) || root >= v.bytes || v.bytes - root < 4096))
        return dv_fail(-EINVAL, "EPT root must be a 4 KiB aligned table inside the arena");
    if (set_dev(c)) return -EIO;
    HIPCHK(hipDeviceSynchronize());
    v.ept_root = root;
    return upload_vms(c);
}

extern "C" int devirt_process_create(devirt_ctx *c, uint32_t vm, uint64_t cr3_gpa, uint32_t levels, uint32_t *asid) {
    if (!c || !asid) return dv_fail(-EINVAL, "NULL argument");
    if (vm >= c->vms.size()) return dv_fail(-ENOENT, "no VM %u", vm);
    if (levels < 3 || levels > 5) return dv_fail(-EINVAL, "levels must be 3 (PAE), 4 or 5");
    if (server_owns(c)) return dv_fail(-EBUSY, "a serving loop owns this context");
    if (c->procs.size() >= 0x7FFFFFFF) return dv_fail(-EINVAL, "too many processes");
    if (set_dev(c)) return -EIO;
    HIPCHK(hipDeviceSynchronize());
    c->procs.push_back(DProc{cr3_gpa, vm, levels});
    int rc = upload_procs(c);
    if (rc) {
        c->procs.pop_back();
        return rc;
    }
    *asid = (uint32_t)(c->procs.size() - 1);
    return 0;
}

DView view_of(const devirt_ctx *c) {
    DView v;
    v.vms = c->d_vms;
    v.procs = c->d_procs;
    v.nvm = (uint32_t)c->vms.size();
    v.nproc = (uint32_t)c->procs.size();
    v.lds = 0;
    v.lds_idx = kLdsNone;
    v.lds_idx_vm = kLdsNone;
    v.pad = 0;
    return v;
}

// ---------------------------------------------------------------- workspaces
static uint64_t default_seg_cap() {
    const char *e = getenv("DEVIRT_SEG_CAP");
    if (e && *e) {
        unsigned long long v = strtoull(e, nullptr, 10);
        if (v >= 64) return v;
    }
    return 8ull << 20;  // 8 Mi segments per queue (256 MiB)
}

Workspace *get_ws(devirt_ctx *c, hipStream_t s) {
    auto it = c->ws.find(s);
    if (it != c->ws.end()) return it->second;
    Workspace *w = new Workspace();
    w->stream = s;
    c->ws[s] = w;
    return w;
}

static bool stream_capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

template <class T>
static int grow(devirt_ctx *c, Workspace *w, T *&p, uint64_t &cap, uint64_t need, const char *what) {
    (void)c;
    if (need <= cap && p) return 0;
    if (stream_capturing(w->stream))
        return dv_fail(-EBUSY, "workspace %s must grow while the stream is being captured; run once uncaptured first",
                       what);
    HIPCHK(hipStreamSynchronize(w->stream));
    for (auto &g : w->graphs) hipGraphExecDestroy(g.exec);
    w->graphs.clear();
    uint64_t ncap = std::max<uint64_t>(need, cap * 2);
    if (ncap < 64) ncap = 64;
    T *np = nullptr;
    if (hipMalloc(&np, ncap * sizeof(T)) != hipSuccess) return dv_fail(-ENOMEM, "hipMalloc workspace %s", what);
    hipFree(p);
    p = np;
    cap = ncap;
    return 0;
}

int ensure_ws(devirt_ctx *c, Workspace *w, uint64_t n_req, uint64_t n_epochs, bool need_pending, uint64_t min_segs) {
    int rc;
    const uint64_t segs = w->segs ? std::max<uint64_t>(w->seg_cap, min_segs) : std::max(default_seg_cap(), min_segs);
    if ((rc = grow(c, w, w->segs, w->seg_cap, segs, "segments"))) return rc;
    if ((rc = grow(c, w, w->shorts, w->short_cap, w->seg_cap, "short segments"))) return rc;
    if ((rc = grow(c, w, w->ctr, w->ctr_cap, std::max<uint64_t>(n_epochs, 1), "epoch counters"))) return rc;
    if ((rc = grow(c, w, w->t0, w->t0_cap, 1, "clock"))) return rc;
    if ((rc = grow(c, w, w->spill, w->spill_cap, std::max<uint64_t>(n_req, 1), "spill list"))) return rc;
    if ((rc = grow(c, w, w->large, w->large_cap, std::max<uint64_t>(n_req, 1), "large list"))) return rc;
    uint64_t tiles = (n_req + kFaultTile - 1) / kFaultTile;
    if ((rc = grow(c, w, w->tiles, w->tiles_cap, std::max<uint64_t>(tiles, 1), "fault tiles"))) return rc;
    if (need_pending && (rc = grow(c, w, w->pending, w->pending_cap, std::max<uint64_t>(n_req, 1), "pending")))
        return rc;
    return 0;
}

DBatch make_batch(devirt_ctx *c, Workspace *w) {
    DBatch b;
    memset(&b, 0, sizeof b);
    if (w) {
        b.segs = w->segs;
        b.shorts = w->shorts;
        b.part_cap = std::min(w->seg_cap, w->short_cap) / kQParts;
        b.spill = w->spill;
        b.large = w->large;
        b.ctr = w->ctr;
        b.pending = w->pending;
        b.t0 = w->t0;
    }
    b.counters = (c->profiling & DEVIRT_PROF_COUNTERS) ? c->d_counters : nullptr;
    b.ns_num = 1000000ull;
    b.ns_den = c->wall_khz;
    b.group = c->cfg.group;
    b.seg_chunks = c->cfg.seg_chunks;
    b.inline_bytes = c->cfg.inline_bytes;
    b.nontemporal = c->cfg.nontemporal;
    b.large_pages = c->cfg.large_pages;
    return b;
}

// ------------------------------------------------------------- profiling
int prof_begin(devirt_ctx *c, hipStream_t s, int kind, ProfEv **out) {
    *out = nullptr;
    if (!(c->profiling & DEVIRT_PROF_TIMING)) return 0;
    ProfEv e;
    e.kind = kind;
    // timing only: no system-scope fence (a cache writeback and invalidate
    // that would be counted in the bracketed kernel's time)
    HIPCHK(hipEventCreateWithFlags(&e.a, hipEventDisableSystemFence));
    HIPCHK(hipEventCreateWithFlags(&e.b, hipEventDisableSystemFence));
    HIPCHK(hipEventRecord(e.a, s));
    c->prof.push_back(e);
    *out = &c->prof.back();
    return 0;
}

int prof_end(devirt_ctx *c, hipStream_t s, ProfEv *e) {
    if (!e) return 0;
    (void)c;
    HIPCHK(hipEventRecord(e->b, s));
    return 0;
}

static int prof_collect(devirt_ctx *c) {
    for (auto &e : c->prof) {
        float ms = 0;
        HIPCHK(hipEventSynchronize(e.b));
        HIPCHK(hipEventElapsedTime(&ms, e.a, e.b));
        if (e.kind == 0) {
            c->stats.copy_ms += ms;
            c->stats.copy_launches++;
        } else {
            c->stats.xlat_ms += ms;
            c->stats.xlat_launches++;
        }
        hipEventDestroy(e.a);
        hipEventDestroy(e.b);
    }
    c->prof.clear();
    return 0;
}

extern "C" int devirt_set_profiling(devirt_ctx *c, int flags) {
    if (!c) return dv_fail(-EINVAL, "ctx is NULL");
    if (flags & ~(DEVIRT_PROF_TIMING | DEVIRT_PROF_COUNTERS)) return dv_fail(-EINVAL, "unknown profiling flags");
    c->profiling = flags;
    return 0;
}

extern "C" int devirt_get_stats(devirt_ctx *c, devirt_stats *out) {
    if (!c || !out) return dv_fail(-EINVAL, "NULL argument");
    if (set_dev(c)) return -EIO;
    HIPCHK(hipDeviceSynchronize());
    int rc = prof_collect(c);
    if (rc) return rc;
    DCounters h;
    HIPCHK(hipMemcpy(&h, c->d_counters, sizeof h, hipMemcpyDeviceToHost));
    *out = c->stats;
    out->pages_walked = h.pages_walked;
    out->cache_hits = h.cache_hits;
    out->cache_misses = h.cache_misses;
    out->segments = h.segments;
    out->inline_segments = h.inline_segments;
    out->ad_atomics = h.ad_atomics;
    out->spilled_groups = h.spilled_groups;
    out->large_requests = h.large_requests;
    return 0;
}

extern "C" int devirt_reset_stats(devirt_ctx *c) {
    if (!c) return dv_fail(-EINVAL, "ctx is NULL");
    if (set_dev(c)) return -EIO;
    HIPCHK(hipDeviceSynchronize());
    int rc = prof_collect(c);
    if (rc) return rc;
    memset(&c->stats, 0, sizeof c->stats);
    HIPCHK(hipMemset(c->d_counters, 0, sizeof(DCounters)));
    return 0;
}

// ------------------------------------------------------------- data path
static int grid_for(devirt_ctx *c, uint64_t waves_needed, uint32_t block, uint32_t per_cu) {
    uint64_t wpb = block / 64;
    uint64_t g = (waves_needed + wpb - 1) / wpb;
    uint64_t cap = (uint64_t)c->cus * per_cu;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (int)g;
}

static int map_run(devirt_ctx *c, MapArgs &a, const devirt_map *maps, uint64_t n, const uint64_t *pool_gpa,
                   const std::vector<uint64_t> &hpa, devirt_result *res, uint64_t *n_used, hipStream_t s);

extern "C" int devirt_map_pages(devirt_ctx *c, uint32_t asid, const devirt_map *maps, uint64_t n,
                                const uint64_t *pool_gpa, uint64_t n_pool, devirt_result *res, uint64_t *n_used,
                                void *stream) {
    if (!c) return dv_fail(-EINVAL, "ctx is NULL");
    if (server_owns(c)) return dv_fail(-EBUSY, "a serving loop owns this context");
    if (n > kMapMax) return dv_fail(-EINVAL, "at most %llu maps per call", (unsigned long long)kMapMax);
    if (!n_used || (n && (!maps || !res)) || (n_pool && !pool_gpa)) return dv_fail(-EINVAL, "NULL argument");
    if (((uintptr_t)maps & 7) || ((uintptr_t)res & 7)) return dv_fail(-EINVAL, "maps and res must be 8-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    if (set_dev(c)) return -EIO;
    std::vector<uint64_t> hpa;
    int rc = dv_map_pool_check(c, asid, pool_gpa, n_pool, hpa);
    if (rc) return rc;
    const bool ept = asid < c->procs.size() && c->vms[c->procs[asid].vm].ept_root != ~0ull;
    MapArgs a;
    a.asid = asid;
    a.ept_pool = ept ? 1 : 0;
    a.ept_map = 0;
    a.vm = 0;
    return map_run(c, a, maps, n, pool_gpa, hpa, res, n_used, s);
}

// The pool of a guest-table map batch: aligned, distinct frames.  For a
// memslot VM each must lie in a memslot, which gives its arena offset in hpa;
// for a VM with an EPT the frames are translated on the device, through the
// EPT (hpa holds zeros).
int dv_map_pool_check(const devirt_ctx *c, uint32_t asid, const uint64_t *pool_gpa, uint64_t n_pool,
                      std::vector<uint64_t> &hpa) {
    hpa.assign(n_pool, 0);
    const bool ept = asid < c->procs.size() && c->vms[c->procs[asid].vm].ept_root != ~0ull;
    if (asid < c->procs.size() && n_pool) {
        // distinct: a strictly ascending pool (the usual case) needs no sort
        bool ascending = true;
        for (uint64_t k = 1; k < n_pool && ascending; ++k) ascending = pool_gpa[k - 1] < pool_gpa[k];
        if (!ascending) {
            std::vector<uint64_t> sorted(pool_gpa, pool_gpa + n_pool);
            std::sort(sorted.begin(), sorted.end());
            if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
                return dv_fail(-EINVAL, "pool frames must be distinct");
        }
        for (uint64_t k = 0; k < n_pool; ++k)
            if (pool_gpa[k] & 0xFFF)
                return dv_fail(-EINVAL, "pool frame %#llx is unaligned", (unsigned long long)pool_gpa[k]);
    }
    if (asid < c->procs.size() && n_pool && !ept) {
        const VmHost &v = c->vms[c->procs[asid].vm];
        std::vector<const VmHost::Slot *> sl;
        for (const auto &x : v.slots)
            if (x.used) sl.push_back(&x);
        std::sort(sl.begin(), sl.end(), [](const VmHost::Slot *p, const VmHost::Slot *q) { return p->gpa < q->gpa; });
        const VmHost::Slot *q = nullptr;  // the slot of the previous frame, tried first
        for (uint64_t k = 0; k < n_pool; ++k) {
            const uint64_t g = pool_gpa[k];
            if (!q || g < q->gpa || g - q->gpa >= q->bytes) {
                // the last slot starting at or below g
                auto it = std::upper_bound(sl.begin(), sl.end(), g,
                                           [](uint64_t x, const VmHost::Slot *r) { return x < r->gpa; });
                q = it == sl.begin() ? nullptr : *(it - 1);
            }
            if (!q || g - q->gpa >= q->bytes)
                return dv_fail(-EINVAL, "pool frame %#llx is outside every memslot", (unsigned long long)g);
            hpa[k] = q->off + (g - q->gpa);
        }
    }
    return 0;
}

// The map launches of devirt_map_pages and devirt_ept_map_pages: workspace,
// pool upload (pool_gpa: the frames as the caller named them; hpa: their
// arena offsets, or zeros for frames the device translates), kernels.
static int map_run(devirt_ctx *c, MapArgs &a, const devirt_map *maps, uint64_t n, const uint64_t *pool_gpa,
                   const std::vector<uint64_t> &hpa, devirt_result *res, uint64_t *n_used, hipStream_t s) {
    const uint64_t n_pool = hpa.size();
    Workspace *w = get_ws(c, s);
    // hash sets of at least twice the entries they can hold
    const uint64_t m = std::min<uint64_t>(4 * n, n_pool);
    auto log2_for = [](uint64_t entries) {
        uint32_t l = 6;
        while ((1ull << l) < 2 * entries) ++l;
        return l;
    };
    const uint32_t tl = log2_for(m + 1), pl = log2_for(n);
    const uint64_t T = 1ull << tl, P = 1ull << pl;
    const uint64_t words = T + m + P + 4 + m + 2 * n_pool;
    int rc;
    if ((rc = grow(c, w, w->map_buf, w->map_cap, words, "map buffers"))) return rc;
    uint64_t *b = w->map_buf;
    a.v = view_of(c);
    a.maps = maps;
    a.n = n;
    a.res = res;
    a.n_used = n_used;
    a.n_pool = n_pool;
    a.tset = b;  // tset, tkeys, pset: cleared to ~0 together; sc: to 0
    a.tset_log2 = tl;
    a.tkeys = b + T;
    a.m = m;
    a.rank = m <= kMapRankMax;
    a.pset = b + T + m;
    a.pset_log2 = pl;
    a.sc = b + T + m + P;
    a.tkeys_sorted = b + T + m + P + 4;
    a.pool_gpa = b + T + 2 * m + P + 4;
    a.pool_hpa = b + T + 2 * m + P + 4 + n_pool;
    if (n_pool) {
        // staged through pinned memory; the previous upload from it must be done
        if (w->map_ev) HIPCHK(hipEventSynchronize(w->map_ev));
        if (w->map_pool_host_cap < 2 * n_pool) {
            hipHostFree(w->map_pool_host);
            w->map_pool_host = nullptr;
            w->map_pool_host_cap = 0;
            HIPCHK(hipHostMalloc((void **)&w->map_pool_host, 2 * n_pool * sizeof(uint64_t), hipHostMallocDefault));
            w->map_pool_host_cap = 2 * n_pool;
        }
        memcpy(w->map_pool_host, pool_gpa, n_pool * sizeof(uint64_t));
        memcpy(w->map_pool_host + n_pool, hpa.data(), n_pool * sizeof(uint64_t));
        HIPCHK(hipMemcpyAsync((void *)a.pool_gpa, w->map_pool_host, 2 * n_pool * sizeof(uint64_t),
                              hipMemcpyHostToDevice, s));
        if (!w->map_ev) HIPCHK(hipEventCreateWithFlags(&w->map_ev, hipEventDisableTiming));
        HIPCHK(hipEventRecord(w->map_ev, s));
    }
    HIPCHK(launch_map(s, a));  // only arena bytes change: captured batch graphs stay valid
    c->xlat_gen++;             // but cached translations may be stale
    return 0;
}

// The pool of an EPT map batch: a VM with an EPT, and aligned, distinct
// arena pages inside its arena.
int dv_ept_pool_check(const devirt_ctx *c, uint32_t vm, const uint64_t *pool_host, uint64_t n_pool) {
    if (vm >= c->vms.size()) return dv_fail(-EINVAL, "no VM %u", vm);
    const VmHost &v = c->vms[vm];
    if (v.ept_root == ~0ull) return dv_fail(-EINVAL, "VM %u has no EPT", vm);
    for (uint64_t k = 0; k < n_pool; ++k)
        if ((pool_host[k] & 0xFFF) || pool_host[k] >= v.bytes || v.bytes - pool_host[k] < 4096)
            return dv_fail(-EINVAL, "pool page %#llx is unaligned or outside the arena",
                           (unsigned long long)pool_host[k]);
    std::vector<uint64_t> sorted(pool_host, pool_host + n_pool);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
        return dv_fail(-EINVAL, "pool pages must be distinct");
    return 0;
}

extern "C" int devirt_ept_map_pages(devirt_ctx *c, uint32_t vm, const devirt_ept_map *maps, uint64_t n,
                                    const uint64_t *pool_host, uint64_t n_pool, devirt_result *res,
                                    uint64_t *n_used, void *stream) {
    if (!c) return dv_fail(-EINVAL, "ctx is NULL");
    if (server_owns(c)) return dv_fail(-EBUSY, "a serving loop owns this context");
    if (vm >= c->vms.size()) return dv_fail(-EINVAL, "no VM %u", vm);
    const VmHost &v = c->vms[vm];
    if (v.ept_root == ~0ull) return dv_fail(-EINVAL, "VM %u has no EPT", vm);
    if (n > kMapMax) return dv_fail(-EINVAL, "at most %llu maps per call", (unsigned long long)kMapMax);
    if (!n_used || (n && (!maps || !res)) || (n_pool && !pool_host)) return dv_fail(-EINVAL, "NULL argument");
    if (((uintptr_t)maps & 7) || ((uintptr_t)res & 7)) return dv_fail(-EINVAL, "maps and res must be 8-byte aligned");
    if (set_dev(c)) return -EIO;
    int rc = dv_ept_pool_check(c, vm, pool_host, n_pool);
    if (rc) return rc;
    std::vector<uint64_t> hpa(pool_host, pool_host + n_pool);
    static_assert(sizeof(devirt_ept_map) == sizeof(devirt_map), "one record layout for both kinds of map");
    MapArgs a;
    a.asid = 0;
    a.ept_pool = 0;
    a.ept_map = 1;
    a.vm = vm;
    return map_run(c, a, (const devirt_map *)maps, n, pool_host, hpa, res, n_used, (hipStream_t)stream);
}

extern "C" int devirt_translate(devirt_ctx *c, uint32_t asid, const uint64_t *gva_dev, uint64_t n, uint32_t flags,
                                devirt_xlat *out_dev, void *stream) {
    if (!c) return dv_fail(-EINVAL, "ctx is NULL");
    if (flags & ~(DEVIRT_XLAT_WRITE | DEVIRT_XLAT_SET_AD)) return dv_fail(-EINVAL, "unknown flags");
    if (server_owns(c)) return dv_fail(-EBUSY, "a serving loop owns this context");
    if (n == 0) return 0;
    if (!gva_dev || !out_dev) return dv_fail(-EINVAL, "NULL buffer");
    if (set_dev(c)) return -EIO;
    hipStream_t s = (hipStream_t)stream;
    const uint32_t block = 256;
    int grid = grid_for(c, (n + 63) / 64, block, 8);
    ProfEv *pe;
    int rc = prof_begin(c, s, 1, &pe);
    if (rc) return rc;
    HIPCHK(launch_xlat(s, grid, block, view_of(c), asid, gva_dev, n, flags, out_dev,
                       (c->profiling & DEVIRT_PROF_COUNTERS) ? c->d_counters : nullptr));
    return prof_end(c, s, pe);
}

// Pages a request touches, 0 when it is empty or not user-canonical for any depth.
static uint64_t pages_of(uint64_t gva, uint64_t len) {
    if (len == 0 || gva >= (1ull << 56) || len > (1ull << 56) - gva) return 0;
    return ((gva + len - 1) >> 12) - (gva >> 12) + 1;
}

static const uint64_t kPlainInlinePages = 16;

int plain_copy(devirt_ctx *c, uint32_t asid, uint64_t gva, uint64_t host, uint64_t len, uint32_t dir,
               devirt_result *res, void *stream, const StaticScratch *st) {
    if (!c) return dv_fail(-EINVAL, "ctx is NULL");
    if (!res) return dv_fail(-EINVAL, "res_dev is NULL");
    if (len >= (1ull << 32)) return dv_fail(-EINVAL, "len must be < 2^32");
    if (server_owns(c)) return dv_fail(-EBUSY, "a serving loop owns this context");
    if (len && !host) return dv_fail(-EINVAL, "NULL host buffer");
    if (set_dev(c)) return -EIO;
    hipStream_t s = (hipStream_t)stream;
    const uint64_t pages = pages_of(gva, len);
    const bool inl = pages <= kPlainInlinePages;
    int rc;
    DBatch b;
    if (st) {
        // the caller's static scratch: nothing is allocated
        if (pages > st->cap)
            return dv_fail(-EINVAL, "the request touches %llu pages; this entry point takes at most %llu",
                           (unsigned long long)pages, (unsigned long long)st->cap);
        b = make_batch(c, nullptr);
        b.segs = st->segs;
        b.shorts = st->shorts;
        b.ctr = st->ctr;
        b.t0 = st->t0;
        b.part_cap = st->cap;
    } else {
        Workspace *w = get_ws(c, s);
        if ((rc = ensure_ws(c, w, 1, 1, false, inl ? 0 : pages))) return rc;
        b = make_batch(c, w);
        // one request: part 0 spans the whole queue, which holds at least one
        // segment per page, so no run overflows it
        b.part_cap = std::min(w->seg_cap, w->short_cap);
    }
    b.res = res;
    if (c->cfg.fifo_entries) {
        b.fifo = c->d_fifo;
        b.fifo_entries = c->cfg.fifo_entries;
        b.xlat_gen = c->xlat_gen;
    }
    devirt_request rq;
    memset(&rq, 0, sizeof rq);
    rq.gva = gva;
    rq.host = host;
    rq.len = (uint32_t)len;
    rq.asid = asid;
    rq.dir = (uint8_t)dir;
    c->stats.plain_calls++;
    HIPCHK(launch_plain(s, view_of(c), b, rq, inl ? 1 : 0));
    if (!inl) {
        ProfEv *pe = nullptr;
        if (!st && (rc = prof_begin(c, s, 0, &pe))) return rc;
        HIPCHK(launch_copy(s, grid_for(c, pages, c->cfg.copy_wg, c->cfg.copy_wgs_per_cu), c->cfg.copy_wg, b, 0));
        if ((rc = prof_end(c, s, pe))) return rc;
    }
    return 0;
}

extern "C" int devirt_copy_from_guest(devirt_ctx *c, uint32_t asid, uint64_t gva, void *dst, uint64_t len,
                                      devirt_result *res, void *stream) {
    return plain_copy(c, asid, gva, (uint64_t)(uintptr_t)dst, len, DEVIRT_FROM_GUEST, res, stream, nullptr);
}
extern "C" int devirt_copy_to_guest(devirt_ctx *c, uint32_t asid, uint64_t gva, const void *src, uint64_t len,
                                    devirt_result *res, void *stream) {
    return plain_copy(c, asid, gva, (uint64_t)(uintptr_t)src, len, DEVIRT_TO_GUEST, res, stream, nullptr);
}

// Enqueue one batch on stream `s` using workspace `w` (no capture logic here).
//
// Translation of an epoch does not depend on the copies of earlier epochs
// (page tables only change in their A/D bits, which are OR-ed, and no request
// touches a page-table frame), so with several epochs the translate launches
// run on a side stream ahead of the copies: translate(e) overlaps copy(e-1).
// The segment queue is split in two halves used by alternate epochs;
// translate(e) waits for copy(e-2), the last user of its half.  Copies stay in
// epoch order on `s`.
//
// Payload bytes move in epoch order: a translate launch that may overlap an
// earlier epoch's copy (overlap on, e >= 1) copies nothing itself.  It gets no
// inline copies, and a group whose runs overflow its queue part goes to the
// epoch's spill list.  The spill pass of epoch e then runs either on the side
// stream after copy(e-1) and before translate(e+1) (spill_side 1), so that it
// overlaps copy(e), which moves bytes of the same epoch (no conflicts; a run
// both move is moved twice with the same bytes), and copy(e+1) waits for it
// through translate(e+1); or on `s` right after copy(e) (spill_side 0).  The
// first keeps every copy launch right behind the previous one; the second
// lets translate(e+1) start ahead of copy(e), which on long copies leaves the
// copy more of the GPU.  The fault list follows the spill passes.
// A small epoch gets smaller groups, so that it still spreads over about 4
// wavefronts per CU (results do not depend on the group).
static uint32_t epoch_group(const devirt_ctx *c, uint64_t n) {
    const uint64_t spread = (n + 4ull * c->cus - 1) / (4ull * c->cus);
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(c->cfg.group, spread));
}

// The spill pass of epoch e (overlap on, e >= 1): the groups of the epoch
// whose runs overflowed their queue part, translated again and copied.
static hipError_t spill_pass(devirt_ctx *c, hipStream_t st, const DView &v, const DBatch &b, const Workspace *w,
                             uint64_t half, const std::vector<uint64_t> &epochs, size_t e) {
    const uint64_t r0 = epochs[e - 1], r1 = epochs[e];
    if (r1 <= r0) return hipSuccess;
    DBatch be = b;
    be.segs = w->segs + (e & 1) * half;
    be.shorts = w->shorts + (e & 1) * half;
    be.part_cap = half / kQParts;
    be.spill_mode = 1;
    be.inline_bytes = 0;
    be.group = epoch_group(c, r1 - r0);
    return launch_spill(st, grid_for(c, (r1 - r0 + be.group - 1) / be.group, c->cfg.xlat_wg, c->cfg.xlat_wgs_per_cu),
                        (int)c->cfg.xlat_wg, v, be, r0, r1, (uint32_t)e);
}

static int enqueue_batch(devirt_ctx *c, Workspace *w, const BatchArgs &a, hipStream_t s) {
    DBatch b = make_batch(c, w);
    b.reqs = a.reqs;
    b.res = a.res;
    b.t_done = a.t_done;
    const DView v = view_of(c);
    const size_t ne = a.epochs.size();
    if (a.direct) {
        // one epoch, every group the first of some wavefront (no claims, so no
        // counter reset), copies by the translating wavefronts: one launch
        b.group = 1;
        HIPCHK(launch_translate_groups(s, grid_for(c, a.n, c->cfg.xlat_wg, 1u << 20), (int)c->cfg.xlat_wg, v, b, 0,
                                       a.n, 0, 1));
        if (a.faults || a.n_faults) {
            uint64_t tiles = (a.n + kFaultTile - 1) / kFaultTile;
            HIPCHK(launch_fault_count(s, a.res, a.n, w->tiles));
            HIPCHK(launch_fault_scan(s, w->tiles, tiles, a.n_faults));
            if (a.faults) HIPCHK(launch_fault_scatter(s, a.res, a.n, w->tiles, a.faults));
        }
        return 0;
    }
    HIPCHK(launch_reset(s, b, (uint32_t)ne));
    const bool overlap = ne > 1 && c->cfg.overlap;
    const bool spill_side = c->cfg.spill_side != 0;
    hipStream_t side = s;
    if (overlap) {
        if (!w->side) HIPCHK(hipStreamCreateWithFlags(&w->side, hipStreamNonBlocking));
        side = w->side;
        while (w->events.size() < 2 * ne + 2) {
            hipEvent_t e;
            HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            w->events.push_back(e);
        }
        HIPCHK(hipEventRecord(w->events[2 * ne], s));  // fork: the side stream starts after the reset
        HIPCHK(hipStreamWaitEvent(side, w->events[2 * ne], 0));
    }
    const uint64_t cap = std::min(w->seg_cap, w->short_cap);
    const uint64_t half = overlap ? cap / 2 : cap;
    uint64_t r0 = 0;
    int rc;
    for (size_t e = 0; e < ne; ++e) {
        const uint64_t r1 = a.epochs[e];
        DBatch be = b;
        be.segs = w->segs + (overlap ? (e & 1) * half : 0);
        be.shorts = w->shorts + (overlap ? (e & 1) * half : 0);
        be.part_cap = half / kQParts;
        be.spill_mode = (overlap && e >= 1) ? 1u : 0u;
        if (be.spill_mode) be.inline_bytes = 0;
        hipEvent_t t_done = overlap ? w->events[2 * e] : nullptr;
        hipEvent_t c_done = overlap ? w->events[2 * e + 1] : nullptr;
        if (overlap && e >= 2 && (spill_side || r1 > r0)) {
            // translate(e) reuses the queue half of copy(e-2); on the side
            // stream the spill pass of epoch e-1 runs after copy(e-2) and
            // translate(e-1), ahead of translate(e), so copy(e) waits for it
            HIPCHK(hipStreamWaitEvent(side, w->events[2 * (e - 2) + 1], 0));
            if (spill_side) HIPCHK(spill_pass(c, side, v, b, w, half, a.epochs, e - 1));
        }
        if (r1 > r0) {
            be.group = epoch_group(c, r1 - r0);
            const uint64_t groups = (r1 - r0 + be.group - 1) / be.group;
            ProfEv *pe;
            if ((rc = prof_begin(c, side, 1, &pe))) return rc;
            HIPCHK(launch_translate_groups(side, grid_for(c, groups, c->cfg.xlat_wg, c->cfg.xlat_wgs_per_cu),
                                           (int)c->cfg.xlat_wg, v, be, r0, r1, (uint32_t)e, 0));
            // the epoch's large requests, a workgroup each (returns at once when there are none)
            if (be.large_pages)
                HIPCHK(launch_translate_large(side, (int)(2ull * c->cus), 256, v, be, r0, (uint32_t)e));
            if ((rc = prof_end(c, side, pe))) return rc;
            if (overlap) {
                HIPCHK(hipEventRecord(t_done, side));
                HIPCHK(hipStreamWaitEvent(s, t_done, 0));
            }
            if ((rc = prof_begin(c, s, 0, &pe))) return rc;
            HIPCHK(launch_copy(s, (int)((uint64_t)c->cus * c->cfg.copy_wgs_per_cu), (int)c->cfg.copy_wg, be,
                               (uint32_t)e));
            if ((rc = prof_end(c, s, pe))) return rc;
        }
        // the spill pass uses no queue: translate(e+2) need not wait for it
        if (overlap) HIPCHK(hipEventRecord(c_done, s));
        if (overlap && !spill_side && e >= 1) HIPCHK(spill_pass(c, s, v, b, w, half, a.epochs, e));
        r0 = r1;
    }
    // the last epoch's spill pass (epochs before it ran theirs ahead of a
    // later translate): after copy(ne-2), under copy(ne-1)
    if (overlap && spill_side) {
        HIPCHK(hipStreamWaitEvent(side, w->events[2 * (ne - 2) + 1], 0));
        HIPCHK(spill_pass(c, side, v, b, w, half, a.epochs, ne - 1));
    }
    // every translate launch is already joined into `s` through its copy's wait
    if (a.faults || a.n_faults) {
        // Every result is final once the last translate launch is done: the
        // copies move bytes only, and a spill pass writes the same results
        // again.  With overlap the fault list is therefore built on the side
        // stream under the last copy, and `s` joins it at the end.
        const hipStream_t fs = overlap && spill_side ? side : s;
        uint64_t tiles = (a.n + kFaultTile - 1) / kFaultTile;
        HIPCHK(launch_fault_count(fs, a.res, a.n, w->tiles));
        HIPCHK(launch_fault_scan(fs, w->tiles, tiles, a.n_faults));
        if (a.faults) HIPCHK(launch_fault_scatter(fs, a.res, a.n, w->tiles, a.faults));
    }
    if (overlap && spill_side) {  // `s` joins the side stream: the last spill pass and the fault list
        HIPCHK(hipEventRecord(w->events[2 * ne + 1], side));
        HIPCHK(hipStreamWaitEvent(s, w->events[2 * ne + 1], 0));
    }
    return 0;
}

static uint64_t hash_key(const std::vector<uint64_t> &k) {
    uint64_t h = 1469598103934665603ull;
    for (uint64_t x : k) {
        h ^= x;
        h *= 1099511628211ull;
        h ^= h >> 29;
    }
    return h;
}

extern "C" int devirt_submit_batch(devirt_ctx *c, const devirt_request *reqs, uint64_t n, const uint64_t *epoch_end,
                                   uint32_t n_epochs, devirt_result *res, devirt_fault *faults, uint64_t *n_faults,
                                   uint64_t *t_done, void *stream) {
    if (!c) return dv_fail(-EINVAL, "ctx is NULL");
    if (server_owns(c)) return dv_fail(-EBUSY, "a serving loop owns this context");
    return dv_submit(c, reqs, n, epoch_end, n_epochs, res, faults, n_faults, t_done, (hipStream_t)stream, true);
}

// Batches of at most this many requests may run as one direct launch.
static constexpr uint64_t kDirectMaxReqs = 64;

int dv_submit(devirt_ctx *c, const devirt_request *reqs, uint64_t n, const uint64_t *epoch_end, uint32_t n_epochs,
              devirt_result *res, devirt_fault *faults, uint64_t *n_faults, uint64_t *t_done, hipStream_t s,
              bool allow_graph, bool allow_direct) {
    if (n && (!reqs || !res)) return dv_fail(-EINVAL, "NULL request or result buffer");
    if (((uintptr_t)reqs & 15) || ((uintptr_t)res & 7)) return dv_fail(-EINVAL, "reqs must be 16-byte aligned");
    BatchArgs a;
    a.reqs = reqs;
    a.n = n;
    a.res = res;
    a.faults = faults;
    a.n_faults = n_faults;
    a.t_done = t_done;
    if (epoch_end) {
        if (n_epochs == 0) return dv_fail(-EINVAL, "n_epochs is 0 with an epoch array");
        uint64_t prev = 0;
        for (uint32_t e = 0; e < n_epochs; ++e) {
            if (epoch_end[e] < prev || epoch_end[e] > n) return dv_fail(-EINVAL, "epoch ends must ascend within [0, n]");
            prev = epoch_end[e];
        }
        if (prev != n) return dv_fail(-EINVAL, "the last epoch must end at n");
        a.epochs.assign(epoch_end, epoch_end + n_epochs);
    } else {
        a.epochs.assign(1, n);
    }
    if (set_dev(c)) return -EIO;
    Workspace *w = get_ws(c, s);
    int rc = ensure_ws(c, w, n, a.epochs.size(), t_done != nullptr, 0);
    if (rc) return rc;
    c->stats.batches++;
    c->stats.epochs += a.epochs.size();
    // the direct launch: one epoch of at most kDirectMaxReqs requests, one
    // request per wavefront, no completion times
    a.direct = allow_direct && a.epochs.size() == 1 && n > 0 && n <= kDirectMaxReqs && !t_done &&
               (uint64_t)grid_for(c, n, c->cfg.xlat_wg, 1u << 20) * (c->cfg.xlat_wg / 64) >= n;
    if (a.direct) return enqueue_batch(c, w, a, s);
    if (!allow_graph || !c->cfg.use_graph || c->profiling || n == 0 || stream_capturing(s))
        return enqueue_batch(c, w, a, s);
    // graph cache: key = every argument that ends up in a kernel parameter
    std::vector<uint64_t> key = {(uint64_t)(uintptr_t)reqs, n, (uint64_t)(uintptr_t)res, (uint64_t)(uintptr_t)faults,
                                 (uint64_t)(uintptr_t)n_faults, (uint64_t)(uintptr_t)t_done, c->tables_version,
                                 c->cfg_version, (uint64_t)(uintptr_t)w->segs, w->seg_cap,
                                 (uint64_t)(uintptr_t)w->shorts, w->short_cap};
    key.insert(key.end(), a.epochs.begin(), a.epochs.end());
    const uint64_t h = hash_key(key);
    for (auto &g : w->graphs) {
        if (g.hash == h && g.key == key) {
            c->stats.graph_replays++;
            HIPCHK(hipGraphLaunch(g.exec, s));
            return 0;
        }
    }
    // Capture on a private non-blocking stream (the legacy null stream cannot be
    // captured), then launch the graph on the caller's stream.
    if (!c->capture_stream) HIPCHK(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
    rc = enqueue_batch(c, w, a, c->capture_stream);
    hipError_t ee = hipStreamEndCapture(c->capture_stream, &graph);
    if (rc) {
        if (graph) hipGraphDestroy(graph);
        return rc;
    }
    if (ee != hipSuccess) return dv_fail(-EIO, "hipStreamEndCapture: %s", hipGetErrorString(ee));
    hipGraphExec_t exec = nullptr;
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (ie != hipSuccess) return dv_fail(-EIO, "hipGraphInstantiate: %s", hipGetErrorString(ie));
    if (w->graphs.size() >= 8) {
        HIPCHK(hipStreamSynchronize(s));
        hipGraphExecDestroy(w->graphs.front().exec);
        w->graphs.erase(w->graphs.begin());
    }
    w->graphs.push_back(GraphEntry{h, key, exec});
    HIPCHK(hipGraphLaunch(exec, s));
    return 0;
}

extern "C" int devirt_sync(devirt_ctx *c, void *stream) {
    if (!c) return dv_fail(-EINVAL, "ctx is NULL");
    if (set_dev(c)) return -EIO;
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    return 0;
}

// ---------------------------------------------------------------- config
extern "C" int devirt_get_config(devirt_ctx *c, devirt_config *cfg) {
    if (!c || !cfg) return dv_fail(-EINVAL, "NULL argument");
    *cfg = c->cfg;
    return 0;
}

extern "C" int devirt_set_config(devirt_ctx *c, const devirt_config *cfg) {
    if (!c || !cfg) return dv_fail(-EINVAL, "NULL argument");
    int rc = check_config(*cfg);
    if (rc) return rc;
    c->cfg = *cfg;
    c->cfg_version++;
    return 0;
}

// Median time of `reps` executions of the batch under the current config.
static int time_batch(devirt_ctx *c, const devirt_request *reqs, uint64_t n, const uint64_t *epoch_end,
                      uint32_t n_epochs, devirt_result *res, devirt_fault *faults, uint64_t *n_faults, void *stream,
                      uint32_t reps, hipEvent_t e0, hipEvent_t e1, double *ms_out) {
    hipStream_t s = (hipStream_t)stream;
    int rc = devirt_submit_batch(c, reqs, n, epoch_end, n_epochs, res, faults, n_faults, nullptr, stream);  // warm-up
    if (rc) return rc;
    std::vector<double> ts;
    for (uint32_t r = 0; r < reps; ++r) {
        HIPCHK(hipEventRecord(e0, s));
        if ((rc = devirt_submit_batch(c, reqs, n, epoch_end, n_epochs, res, faults, n_faults, nullptr, stream)))
            return rc;
        HIPCHK(hipEventRecord(e1, s));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        ts.push_back(ms);
    }
    std::sort(ts.begin(), ts.end());
    *ms_out = ts[ts.size() / 2];
    return 0;
}

// Coordinate descent over the launch knobs: each knob in turn is set to each
// of its candidate values, with the others at the best found so far.
extern "C" int devirt_autotune(devirt_ctx *c, const devirt_request *reqs, uint64_t n, const uint64_t *epoch_end,
                               uint32_t n_epochs, devirt_result *res, devirt_fault *faults, uint64_t *n_faults,
                               void *stream, uint32_t reps, devirt_config *best, double *best_ms) {
    if (!c) return dv_fail(-EINVAL, "ctx is NULL");
    if (reps == 0) reps = 3;
    if (set_dev(c)) return -EIO;
    const devirt_config base = c->cfg;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const int prof = c->profiling;
    c->profiling = 0;
    devirt_config cur = base;
    double cur_ms = 0;
    c->cfg_version++;
    int rc = time_batch(c, reqs, n, epoch_end, n_epochs, res, faults, n_faults, stream, reps, e0, e1, &cur_ms);
    typedef void (*Setter)(devirt_config &, uint32_t);
    struct Knob {
        Setter set;
        std::vector<uint32_t> values;
    };
    // Overlap first: the best group size depends on whether translation
    // shares the GPU with the copies.  Without overlap the translate grid is
    // the 3 workgroups of 256 per CU that its registers allow.
    const std::vector<Knob> knobs = {
        {[](devirt_config &k, uint32_t v) {
             k.overlap = v ? 1 : 0;
             k.xlat_wgs_per_cu = v ? v : 3;
         },
         {0, 1, 2}},
        {[](devirt_config &k, uint32_t v) { k.group = v; }, {8, 16, 32, 64}},
        {[](devirt_config &k, uint32_t v) { k.copy_wg = v; }, {256, 512, 1024}},
        {[](devirt_config &k, uint32_t v) { k.copy_wgs_per_cu = v; }, {4, 8, 16, 32, 64}},
        {[](devirt_config &k, uint32_t v) { k.seg_chunks = v; }, {1, 2, 4, 16, 64}},
        {[](devirt_config &k, uint32_t v) { k.large_pages = v; }, {0, 64, 128, 256, 1024}},
        {[](devirt_config &k, uint32_t v) { k.spill_side = v; }, {1, 0}},
    };
    for (const auto &kn : knobs) {
        if (rc) break;
        devirt_config keep = cur;
        for (uint32_t v : kn.values) {
            devirt_config k = keep;
            kn.set(k, v);
            if (memcmp(&k, &keep, sizeof k) == 0) continue;
            if (check_config(k)) continue;
            c->cfg = k;
            c->cfg_version++;
            double ms = 0;
            if ((rc = time_batch(c, reqs, n, epoch_end, n_epochs, res, faults, n_faults, stream, reps, e0, e1, &ms)))
                break;
            if (ms < cur_ms) {
                cur_ms = ms;
                cur = k;
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    c->profiling = prof;
    c->cfg = rc ? base : cur;
    c->cfg_version++;
    if (rc) return rc;
    if (best) *best = cur;
    if (best_ms) *best_ms = cur_ms;
    return 0;
}

// ------------------------------------------------------- tuning cache
// One JSON object per line:
//   {"key": "<device>|<workload key>", "ms": <median ms>, "config": {"group": 64, ...}}
// <device> is the architecture name and the CU count.  The last line with a
// key wins; lines that do not parse are skipped.
struct CfgField {
    const char *name;
    uint32_t devirt_config::*field;
};
static const CfgField kCfgFields[] = {
    {"group", &devirt_config::group},
    {"seg_chunks", &devirt_config::seg_chunks},
    {"xlat_wg", &devirt_config::xlat_wg},
    {"xlat_wgs_per_cu", &devirt_config::xlat_wgs_per_cu},
    {"copy_wg", &devirt_config::copy_wg},
    {"copy_wgs_per_cu", &devirt_config::copy_wgs_per_cu},
    {"nontemporal", &devirt_config::nontemporal},
    {"inline_bytes", &devirt_config::inline_bytes},
    {"use_graph", &devirt_config::use_graph},
    {"overlap", &devirt_config::overlap},
    {"fifo_entries", &devirt_config::fifo_entries},
    {"large_pages", &devirt_config::large_pages},
    {"spill_side", &devirt_config::spill_side},
};

static std::string device_key(devirt_ctx *c) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, c->device) != hipSuccess) return std::string();
    char buf[320];
    snprintf(buf, sizeof buf, "%s/%dcu", p.gcnArchName, p.multiProcessorCount);
    return std::string(buf);
}

// Parses one cache line; true when it names `key` and holds a valid config.
static bool parse_tune_line(const std::string &line, const std::string &key, devirt_config *cfg, double *ms) {
    const std::string kk = "\"key\": \"";
    size_t a = line.find(kk);
    if (a == std::string::npos) return false;
    a += kk.size();
    size_t b = line.find('"', a);
    if (b == std::string::npos || line.compare(a, b - a, key) != 0 || b - a != key.size()) return false;
    size_t m = line.find("\"ms\": ", b);
    if (m == std::string::npos) return false;
    *ms = strtod(line.c_str() + m + 6, nullptr);
    devirt_config k = default_config();  // a field the line lacks (written before it existed) keeps its default
    for (const CfgField &f : kCfgFields) {
        const std::string name = std::string("\"") + f.name + "\": ";
        size_t p = line.find(name, m);
        if (p != std::string::npos) k.*(f.field) = (uint32_t)strtoul(line.c_str() + p + name.size(), nullptr, 10);
    }
    if (check_config(k)) return false;
    *cfg = k;
    return true;
}

extern "C" int devirt_autotune_cached(devirt_ctx *c, const char *cache_path, const char *workload_key,
                                      const devirt_request *reqs, uint64_t n, const uint64_t *epoch_end,
                                      uint32_t n_epochs, devirt_result *res, devirt_fault *faults, uint64_t *n_faults,
                                      void *stream, uint32_t reps, devirt_config *best, double *best_ms, int *hit) {
    if (!c || !cache_path || !workload_key) return dv_fail(-EINVAL, "NULL argument");
    if (strchr(workload_key, '"') || strchr(workload_key, '\\') || strchr(workload_key, '\n'))
        return dv_fail(-EINVAL, "workload key must not hold quotes, backslashes or newlines");
    if (set_dev(c)) return -EIO;
    const std::string dev = device_key(c);
    if (dev.empty()) return dv_fail(-EIO, "hipGetDeviceProperties failed");
    const std::string key = dev + "|" + workload_key;
    devirt_config found;
    double found_ms = 0;
    bool have = false;
    if (FILE *f = fopen(cache_path, "r")) {
        char buf[4096];
        while (fgets(buf, sizeof buf, f)) {
            devirt_config k;
            double ms;
            if (parse_tune_line(buf, key, &k, &ms)) {
                found = k;
                found_ms = ms;
                have = true;
            }
        }
        fclose(f);
    }
    if (hit) *hit = have ? 1 : 0;
    if (have) {
        int rc = devirt_set_config(c, &found);
        if (rc) return rc;
        if (best) *best = found;
        if (best_ms) *best_ms = found_ms;
        return 0;
    }
    devirt_config k;
    double ms = 0;
    int rc = devirt_autotune(c, reqs, n, epoch_end, n_epochs, res, faults, n_faults, stream, reps, &k, &ms);
    if (rc) return rc;
    if (best) *best = k;
    if (best_ms) *best_ms = ms;
    std::string line = "{\"key\": \"" + key + "\", \"ms\": ";
    char num[64];
    snprintf(num, sizeof num, "%.6f", ms);
    line += num;
    line += ", \"config\": {";
    bool first = true;
    for (const CfgField &f : kCfgFields) {
        snprintf(num, sizeof num, "%s\"%s\": %u", first ? "" : ", ", f.name, k.*(f.field));
        line += num;
        first = false;
    }
    line += "}}\n";
    FILE *f = fopen(cache_path, "a");
    if (!f) return dv_fail(-EIO, "cannot append to the tuning cache %s", cache_path);
    const bool ok = fputs(line.c_str(), f) >= 0;
    if (fclose(f) != 0 || !ok) return dv_fail(-EIO, "cannot write the tuning cache %s", cache_path);
    return 0;
}

// ------------------------------------------------- translation caches
extern "C" int devirt_fifo_counts(devirt_ctx *c, uint32_t asid, uint64_t *hits, uint64_t *misses) {
    if (!c || !hits || !misses) return dv_fail(-EINVAL, "NULL argument");
    if (asid >= c->procs.size()) return dv_fail(-ENOENT, "no process %u", asid);
    if (server_owns(c)) return dv_fail(-EBUSY, "a serving loop owns this context");
    if (set_dev(c)) return -EIO;
    HIPCHK(hipDeviceSynchronize());
    DFifo f;
    HIPCHK(hipMemcpy(&f, c->d_fifo + asid, sizeof f, hipMemcpyDeviceToHost));
    *hits = f.hits;
    *misses = f.misses;
    return 0;
}

extern "C" int devirt_fifo_flush(devirt_ctx *c) {
    if (!c) return dv_fail(-EINVAL, "ctx is NULL");
    if (server_owns(c)) return dv_fail(-EBUSY, "a serving loop owns this context");
    if (set_dev(c)) return -EIO;
    HIPCHK(hipDeviceSynchronize());
    if (c->d_fifo) HIPCHK(hipMemset(c->d_fifo, 0, c->d_procs_cap * sizeof(DFifo)));
    c->xlat_gen++;
    return 0;
}
