// Internal layouts shared by the host runtime and the gfx950 kernels.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

#include "../../include/devirt.h"

namespace dv {

// x86-64 entry bits (section 4.2 walks the guest's own tables).
constexpr uint64_t kAddrMask = 0x000FFFFFFFFFF000ull;  // address bits 51:12
constexpr uint64_t kP = 1ull, kRW = 2ull, kUS = 4ull, kA = 0x20ull, kD = 0x40ull, kPS = 0x80ull;
// PAE (section 6.2): reserved bits of a root (page-directory-pointer) entry,
// bits 63:52, 8:5 and 2:1, and of a PDE or PTE, bits 62:52.
constexpr uint64_t kPaeRootRsvd = 0xFFF00000000001E6ull;
constexpr uint64_t kPaeRsvd = 0x7FF0000000000000ull;

// A memslot as the device sees it: sorted by gpa, end = gpa + bytes.
struct DSlot {
    uint64_t gpa;
    uint64_t end;
    uint64_t arena_off;
};

// Per-VM device view.  `index` holds one word per 2 MiB of guest-physical
// space below index_len * 2 MiB:
//   0                 no slot overlaps the block
//   delta | 2         one slot covers the whole block; hpa = gpa + delta
//                     (delta = arena_off - slot gpa, 4 KiB aligned, mod 2^64)
//   1                 the block is split between slots / holes: search slots
// When index_complete is set, no slot lies at or above index_len * 2 MiB.
struct DVm {
    uint8_t *arena;
    uint64_t arena_bytes;
    const uint64_t *index;
    const DSlot *slots;
    uint32_t index_len;
    uint32_t nslots;
    uint32_t index_complete;
    uint32_t lds_base;  // kernels: this VM's first slot in the workgroup's LDS copy (kLdsNone: use HBM)
    uint64_t ept_root;  // arena offset of the EPT's level-4 table; kNoEpt: memslots translate
    uint32_t lds_idx;   // kernels: this VM's 2 MiB index in LDS, in 32-bit words (kLdsNone: none)
    uint32_t pad;
};
constexpr uint32_t kLdsNone = 0xFFFFFFFFu;
constexpr uint64_t kNoEpt = ~0ull;

struct DProc {
    uint64_t cr3;
    uint32_t vm;
    uint32_t levels;
};

struct DView {
    const DVm *vms;
    const DProc *procs;
    uint32_t nvm;
    uint32_t nproc;
    uint32_t lds;      // kernels: the VMs' memslots are in the workgroup's LDS (set by the kernel)
    uint32_t lds_idx;  // kernels: first LDS word of VM lds_idx_vm's 2 MiB index (kLdsNone: none)
    uint32_t lds_idx_vm;
    uint32_t pad;
};

// One queued copy segment (32 B): a run of pages of one request whose guest
// side is contiguous in the arena.
struct DSeg {
    uint64_t src;
    uint64_t dst;
    uint32_t len;
    uint32_t req;
    uint64_t pad;
};

// Runs of at most this many bytes go to the short-segment queue, whose
// segments are copied four to a wavefront (one per 16 lanes): one pass of a
// 16-lane group moves 4 x 16 x 16 B = 1 KiB.
constexpr uint32_t kShortRun = 1024;

// Same-address atomics serialise: with one shared counter of queued
// segments the reservation atomics dominated the translate time.  So each
// segment queue is split into kQParts equal parts with a counter each, every
// counter on a 128-byte line of its own, and a translating wavefront appends
// to part (its global index mod kQParts).
constexpr uint32_t kQParts = 32;
constexpr uint32_t kLineWords = 32;

// Per-epoch device counters (word 0 of each line is used).  A segment count
// may exceed its part's capacity; segments past it were either copied by the
// translating wavefront or, when that wavefront may run during an earlier
// epoch's copies, left to the epoch's spill pass (DBatch::spill_mode).
struct DEpochCtr {
    uint32_t group_cursor;  // groups claimed beyond each wavefront's first
    uint32_t pad[kLineWords - 1];
    // segments in part p of the long queue (q[p]) and of the short queue
    // (q[kQParts + p])
    uint32_t q[2 * kQParts][kLineWords];
    uint32_t spill_n;  // groups on the epoch's spill list
    uint32_t pad2[kLineWords - 1];
    uint32_t large_n;  // requests on the epoch's large list
    uint32_t pad3[kLineWords - 1];
};
// A spill-list entry naming one (large) request rather than a group.
constexpr uint64_t kSpillOne = 1ull << 63;
static_assert(2 * kQParts == 64, "one counter per lane of a wavefront");

// A process's translation cache on the per-request path (section 4.2: the
// backend caches translations per guest process in a small FIFO).  Slot i
// holds virtual page vpn[i] at arena offset hpa[i]; bit i of `written` marks
// an entry filled or refreshed by a write.  Entries are valid only while
// `gen` equals the context's translation generation, which every change to
// guest memory or the translation setup advances (A/D bits a hit relies on
// may have been cleared).  hits/misses count lookups since the last flush.
constexpr uint32_t kFifoMax = 16;
struct DFifo {
    uint64_t vpn[kFifoMax];
    uint64_t hpa[kFifoMax];
    uint32_t written;
    uint32_t n;
    uint32_t head;
    uint32_t pad;
    uint64_t gen;
    unsigned long long hits;
    unsigned long long misses;
    uint64_t pad2[3];
};
static_assert(sizeof(DFifo) == 320, "DFifo layout");

// Device counters gathered while profiling.
struct DCounters {
    unsigned long long pages_walked;
    unsigned long long cache_hits;
    unsigned long long cache_misses;
    unsigned long long segments;
    unsigned long long inline_segments;
    unsigned long long ad_atomics;
    unsigned long long spilled_groups;
    unsigned long long large_requests;
};

// Everything one batch launch needs besides the view.
struct DBatch {
    const devirt_request *reqs;
    devirt_result *res;
    uint64_t *t_done;         // may be null
    uint32_t *pending;        // per request, queued segments not yet copied (t_done only)
    DSeg *segs;               // long segments
    DSeg *shorts;             // short segments (len <= kShortRun)
    uint64_t part_cap;        // segments per queue part (a batch uses kQParts parts of each
                              // queue; a per-request call only part 0, as large as the queue)
    // Groups whose segments did not all fit their queue part.  With spill_mode
    // set, translation may run while an earlier epoch is still being copied, so
    // a translating wavefront must not move payload bytes: it puts its group's
    // first request index on the spill list instead (slots [r0, r1) of the
    // epoch's requests; a group appears at most once), and the spill pass,
    // launched after the epoch's copy, translates those groups again and copies
    // all of their runs.  Without spill_mode the wavefront copies them itself.
    uint64_t *spill;
    uint32_t spill_mode;
    // Requests of more than large_pages pages (0: none) are walked by a
    // workgroup in k_translate_large; k_translate_groups lists them in slots
    // [r0, r1) of `large` (the epoch's requests).
    uint32_t large_pages;
    uint64_t *large;
    DEpochCtr *ctr;           // per epoch
    DCounters *counters;      // null unless profiling
    uint64_t *t0;             // device wall clock at batch start
    uint64_t ns_num;          // ns = ticks * ns_num / ns_den
    uint64_t ns_den;
    uint32_t group;
    uint32_t seg_chunks;
    uint32_t inline_bytes;
    uint32_t nontemporal;
    // per-request path only: the processes' translation caches (null: off)
    DFifo *fifo;
    uint64_t xlat_gen;
    uint32_t fifo_entries;
    uint32_t pad1;
};

// ---- launchers (kernels.hip) ------------------------------------------------
hipError_t launch_reset(hipStream_t s, DBatch b, uint32_t n_epochs);
hipError_t launch_translate_groups(hipStream_t s, int grid, int block, DView v, DBatch b, uint64_t r0,
                                   uint64_t r1, uint32_t epoch, int direct);
hipError_t launch_translate_large(hipStream_t s, int grid, int block, DView v, DBatch b, uint64_t r0,
                                  uint32_t epoch);
hipError_t launch_copy(hipStream_t s, int grid, int block, DBatch b, uint32_t epoch);
hipError_t launch_spill(hipStream_t s, int grid, int block, DView v, DBatch b, uint64_t r0, uint64_t r1,
                        uint32_t epoch);
hipError_t launch_plain(hipStream_t s, DView v, DBatch b, devirt_request req, int inline_copy);
hipError_t launch_xlat(hipStream_t s, int grid, int block, DView v, uint32_t asid, const uint64_t *gva,
                       uint64_t n, uint32_t flags, devirt_xlat *out, DCounters *counters);
hipError_t launch_fault_count(hipStream_t s, const devirt_result *res, uint64_t n, uint32_t *tile_cnt);
hipError_t launch_fault_scan(hipStream_t s, uint32_t *tile_cnt, uint64_t ntiles, uint64_t *n_faults);
hipError_t launch_fault_scatter(hipStream_t s, const devirt_result *res, uint64_t n, const uint32_t *tile_off,
                                devirt_fault *faults);
constexpr int kFaultTile = 1024;

// devirt_map_pages: device buffers and arguments of one call.
constexpr uint64_t kMapMax = 1ull << 19;      // maps per call
constexpr int kMapIdxBits = 19;               // map index bits in a page-set slot
constexpr uint64_t kMapRankMax = 1ull << 14;  // longest key list sorted by rank in LDS tiles
struct MapArgs {
    DView v;
    uint32_t asid;
    const devirt_map *maps;
    uint64_t n;
    devirt_result *res;
    uint64_t *n_used;
    uint64_t n_pool;
    const uint64_t *pool_gpa;             // device, n_pool
    uint64_t *pool_hpa;                   // device, n_pool: from the host, or (ept_pool) from k_map_pool
    int ept_pool;                         // the VM has an EPT: pool frames are translated on the device
    // EPT maps (devirt_ept_map_pages): the maps name guest-physical pages of
    // VM `vm` and the arena pages behind them, and the writes go to its EPT;
    // the pool holds arena offsets (pool_gpa == pool_hpa)
    int ept_map;
    uint32_t vm;
    // the tables the batch lacks: a hash set of their keys (tset_log2 slots),
    // the distinct keys in insertion order (m = min(4n, n_pool) slots), sorted
    uint64_t *tset;
    uint32_t tset_log2;
    uint64_t *tkeys, *tkeys_sorted;
    uint64_t m;
    int rank;                             // sort by rank (m <= kMapRankMax), else tiles and merges
    // pages: a hash set of (page << kMapIdxBits | highest map index), ~0 when empty
    uint64_t *pset;
    uint32_t pset_log2;
    uint64_t *sc;                         // 4 scalars
};
hipError_t launch_map(hipStream_t s, const MapArgs &a);

}  // namespace dv
