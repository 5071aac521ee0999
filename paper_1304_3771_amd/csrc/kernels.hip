// gfx950 kernels of the guest-memory translate-and-copy path.
//
// The operation (section 4.2 of the paper): a buffer at a guest virtual
// address is translated page by page -- a software walk of the guest's page
// tables (x86-64 4- or 5-level, or the 32-bit PAE format of the paper's
// prototype, section 6.2) to a guest-physical address, then the VM's memslots
// to the host address (KVM style), or, for a VM described by an extended page
// table, a second software walk of that EPT (the paper's path for other
// hypervisors) -- and its bytes are copied between the guest memory image
// ("arena") and a host buffer.  A fault ends the operation with everything
// before the faulting byte copied, so the operation can be re-executed
// (section 6.6).
//
// Work decomposition (wave64 throughout):
//   translate  one wavefront owns a group of consecutive requests.  A wave
//              prefix sum over their page counts flattens the group's pages;
//              each pass gives every lane one page.  Lanes that start a 2 MiB
//              region ("heads") resolve the upper levels -- the levels above
//              2 through a per-wavefront LDS cache of 1 GiB regions, level 2
//              by a load -- and hand the result to the rest of the region with
//              cross-lane shuffles; every lane then reads its own leaf entry,
//              so neighbouring lanes read neighbouring PTEs in one cache line.
//              Because a group's pages are walked in order, the first fault
//              of each request is exact (ballot + find-first-set) before any
//              side effect: A/D bits are OR-ed only into entries on the paths
//              of pages that will be copied.  Copy segments (runs of pages
//              whose guest side is contiguous in the arena) are appended to a
//              long or a short queue, each split into parts with a counter of
//              their own, with one wave-aggregated atomic per pass and queue.
//   copy       a wavefront takes each long segment, a 16-lane quarter each
//              short one; stores are 16-byte aligned, the source misalignment
//              is absorbed with one neighbour dword and a byte funnel shift,
//              never with a read-modify-write of bytes outside the segment.
//   faults     the ordered fault list is a tile count, a single-workgroup
//              scan and a ballot/mbcnt scatter.
//   map pages  one lane per map walks the tables as they are; device hash
//              sets collect the distinct tables the batch lacks and the last
//              map of each page; the new tables are ordered by rank in LDS
//              tiles (long lists: tiles, then merge rounds), zeroed,
//              linked, and the leaves written -- four launches.
#include <cstring>

#include "dv_internal.h"

namespace dv {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
// Global-address-space views: the copy path and the table walks address HBM
// through integers, so without these the compiler emits flat instructions
// (which also count against the LDS counter and serialise with shuffles).
// (The host compilation pass only parses device functions; it gets no qualifier.)
#if defined(__HIP_DEVICE_COMPILE__)
#define DV_GLOBAL __attribute__((address_space(1)))
#else
#define DV_GLOBAL
#endif
typedef DV_GLOBAL u32x4 g_u32x4;
typedef DV_GLOBAL uint8_t g_u8;
typedef DV_GLOBAL uint64_t g_u64;
typedef DV_GLOBAL unsigned int g_u32;

template <class T>
__device__ __forceinline__ T *gp(uint64_t a) {
    return (T *)(uintptr_t)a;
}
template <class T, class P>
__device__ __forceinline__ T *gp(P *a) {
    return (T *)(uintptr_t)a;
}

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kCacheWays = 16;  // 1 GiB-region cache entries per wavefront

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t mask_le(int lane) {
    return lane >= 63 ? ~0ull : ((2ull << lane) - 1ull);
}
__device__ __forceinline__ uint64_t mask_lt(int lane) { return lane <= 0 ? 0ull : ((1ull << lane) - 1ull); }

__device__ __forceinline__ uint32_t uniform_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
    uint32_t lo = uniform_u32((uint32_t)x), hi = uniform_u32((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl64(uint64_t x, int src) {
    return __shfl((unsigned long long)x, src);
}
__device__ __forceinline__ uint32_t shfl32(uint32_t x, int src) { return (uint32_t)__shfl((int)x, src); }

__device__ __forceinline__ uint64_t load_entry(const uint8_t *arena, uint64_t off) {
    return *gp<const g_u64>(arena + off);
}

// OR bits into the low dword of a page-table entry (A and D live in bits 5, 6).
__device__ __forceinline__ void or_entry(uint8_t *arena, uint64_t off, uint32_t bits) {
    __hip_atomic_fetch_or(gp<g_u32>(arena + off), bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t now_ns(const DBatch &b) {
    uint64_t t = wall_clock64();
    uint64_t t0 = *b.t0;
    return (t - t0) * b.ns_num / b.ns_den;
}

// ------------------------------------------------------------------ memslots
// The translate kernels keep a copy of every VM's sorted memslots in LDS when
// they fit (at most kLdsVms VMs, kLdsSlots slots in all: 12 KiB).  A walk looks
// a memslot up for every table it reads and for the data page; from LDS that
// is a few LDS reads instead of a dependent load of the 2 MiB index.
constexpr uint32_t kLdsSlots = 512;
constexpr uint32_t kLdsVms = 64;
__shared__ DSlot g_lds_slot[kLdsSlots];
__shared__ uint32_t g_lds_off[kLdsVms + 1];

// A VM's 2 MiB index in the LDS area after the slots (from word w0), when it
// fits: one 32-bit word per block, a block inside one slot as (arena_off -
// gpa) / 4 KiB << 2 | 2 (that difference must fit 30 signed bits), a block
// split between slots as 1, a block without a slot as 0.  Entered by every
// thread; ends with a barrier.  Returns (uniformly) w0, or kLdsNone.
typedef DV_GLOBAL DVm g_dvm;
__device__ uint32_t lds_index_load(const g_dvm *vm, uint32_t w0) {
    const uint32_t nblk = vm->index_len;
    const bool fits = vm->ept_root == kNoEpt && nblk > 0 && w0 + nblk <= kLdsSlots * (uint32_t)(sizeof(DSlot) / 4);
    int bad = 0;
    if (fits) {
        uint32_t *words = (uint32_t *)g_lds_slot + w0;
        for (uint32_t b = threadIdx.x; b < nblk; b += blockDim.x) {
            const uint64_t e = gp<const g_u64>(vm->index)[b];
            uint32_t x = (uint32_t)(e & 1u);
            if (e & 2) {
                const int64_t dp = (int64_t)(e & ~0xFFFull) >> 12;
                if (dp < -(1ll << 29) || dp >= (1ll << 29)) bad = 1;
                x = ((uint32_t)(int32_t)dp << 2) | 2u;
            }
            words[b] = x;
        }
    }
    bad = __syncthreads_or(bad);
    return fits && !bad ? w0 : kLdsNone;
}

// Fills the workgroup's copy with VM `one`'s slots only (at LDS slot 0),
// followed by its 2 MiB index when that fits (V.lds_idx, V.lds_idx_vm);
// entered by every thread.  Returns (uniformly) whether the slots are in LDS.
__device__ bool lds_slots_load_one(DView &V, uint32_t one) {
    V.lds_idx = kLdsNone;
    if (one >= V.nvm) return false;
    typedef DV_GLOBAL DSlot g_slot;
    const g_dvm *vm = gp<const g_dvm>(V.vms) + one;
    const uint32_t ns = vm->nslots;
    if (ns > kLdsSlots || one > kLdsVms) return false;
    if (threadIdx.x == 0) g_lds_off[one] = 0;
    for (uint32_t t = threadIdx.x; t < ns; t += blockDim.x) g_lds_slot[t] = gp<const g_slot>(vm->slots)[t];
    V.lds_idx = lds_index_load(vm, ns * (uint32_t)(sizeof(DSlot) / 4));
    V.lds_idx_vm = one;
    return true;
}

// Fills the workgroup's copy; entered by every thread.  Returns (uniformly)
// whether the slots are in LDS.
__device__ bool lds_slots_load(const DView &V) {
    if (V.nvm > kLdsVms) return false;
    typedef DV_GLOBAL DVm g_vm;
    typedef DV_GLOBAL DSlot g_slot;
    const g_vm *vms = gp<const g_vm>(V.vms);
    if (threadIdx.x < 64) {  // one wavefront: exclusive prefix sum of the slot counts
        const uint32_t lane = threadIdx.x;
        const uint32_t cnt = lane < V.nvm ? vms[lane].nslots : 0u;
        uint32_t incl = cnt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t t = (uint32_t)__shfl((int)incl, lane >= (uint32_t)d ? (int)lane - d : (int)lane);
            if (lane >= (uint32_t)d) incl += t;
        }
        if (lane < V.nvm) g_lds_off[lane] = incl - cnt;
        if (lane == V.nvm - 1) g_lds_off[V.nvm] = incl;
        if (V.nvm == 0 && lane == 0) g_lds_off[0] = 0;
    }
    __syncthreads();
    const uint32_t total = g_lds_off[V.nvm];
    if (total > kLdsSlots) return false;
    for (uint32_t t = threadIdx.x; t < total; t += blockDim.x) {
        uint32_t vm = 0;
        while (vm + 1 < V.nvm && g_lds_off[vm + 1] <= t) ++vm;
        g_lds_slot[t] = gp<const g_slot>(vms[vm].slots)[t - g_lds_off[vm]];
    }
    __syncthreads();
    return true;
}

// A VM's table entry as a translate kernel uses it (lds: its slots are in LDS).
__device__ __forceinline__ DVm load_vm(const DView &V, uint32_t vm, bool lds) {
    DVm v = gp<const DV_GLOBAL DVm>(V.vms)[vm];
    v.lds_base = lds ? g_lds_off[vm] : kLdsNone;
    v.lds_idx = lds && vm == V.lds_idx_vm ? V.lds_idx : kLdsNone;
    return v;
}

// GPA -> arena offset (section 4.2: the guest-physical address is turned into
// the host address backing it, as KVM does with its memslots).
__device__ __forceinline__ bool slot_lookup(const DVm &v, uint64_t gpa, uint64_t &hpa) {
    if (v.lds_idx != kLdsNone) {  // the 2 MiB index in LDS: one read unless the block is split
        const uint64_t blk = gpa >> 21;
        if (blk < v.index_len) {
            const uint32_t e = ((const uint32_t *)g_lds_slot)[v.lds_idx + blk];
            if (e & 2) {
                hpa = gpa + ((uint64_t)(int64_t)((int32_t)e >> 2) << 12);
                return true;
            }
            if (!(e & 1)) return false;
        } else if (v.index_complete) {
            return false;
        }
    }
    if (v.lds_base != kLdsNone) {  // binary search of the LDS copy
        const DSlot *sl = g_lds_slot + v.lds_base;
        uint32_t lo = 0, hi = v.nslots;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (sl[mid].gpa <= gpa)
                lo = mid + 1;
            else
                hi = mid;
        }
        if (lo == 0 || gpa >= sl[lo - 1].end) return false;
        hpa = sl[lo - 1].arena_off + (gpa - sl[lo - 1].gpa);
        return true;
    }
    uint64_t blk = gpa >> 21;
    if (blk < v.index_len) {
        uint64_t e = gp<const g_u64>(v.index)[blk];
        if (e & 2) {
            hpa = gpa + (e & ~0xFFFull);
            return true;
        }
        if (!(e & 1)) return false;
    } else if (v.index_complete) {
        return false;
    }
    typedef DV_GLOBAL DSlot g_slot;
    const g_slot *slots = gp<const g_slot>(v.slots);
    uint32_t lo = 0, hi = v.nslots;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (slots[mid].gpa <= gpa)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (lo == 0) return false;
    DSlot s = slots[lo - 1];
    if (gpa >= s.end) return false;
    hpa = s.arena_off + (gpa - s.gpa);
    return true;
}

// ------------------------------------------------------------------ EPT
// Hypervisors other than KVM finish the translation with a second software
// walk, of the extended page table that describes the guest-physical space
// (section 4.2; EPT in section 2.2).  The EPT is 4-level and lives in the
// arena; entry addresses are arena offsets.  Per level, top-down: not
// present (bits 2:0 clear) is a violation; write without read, or any of
// bits 7:3 in a table entry, is a misconfiguration; read and write are
// AND-ed down the walk.  At the leaf: a memory type of 2, 3 or 7, reserved
// bits of a large leaf, or a page outside the arena is a misconfiguration,
// then a missing permission is a violation.  Addresses at or above 2^48 are
// violations.  Every table and page the walk yields lies inside the arena.
constexpr uint32_t kNeedR = 1, kNeedW = 2, kNeedTable = 3;  // a guest table frame may take A/D writes

struct XRes {
    uint64_t hpa;
    uint32_t code;
};

// Inlined: out of line, the call convention costs the translate kernels a
// wave of occupancy even when no VM has an EPT.
__device__ __forceinline__ XRes ept_walk(uint8_t *arena, uint64_t arena_bytes, uint64_t root, uint64_t gpa,
                                      uint32_t need) {
    XRes r{0, DEVIRT_EPT_VIOLATION};
    if (gpa >> 48) return r;
    uint64_t table = root;
    uint64_t perm = 3;
    for (int lvl = 4; lvl >= 1; --lvl) {
        const uint32_t sh = 12u + 9u * (uint32_t)(lvl - 1);
        const uint64_t e = load_entry(arena, table + 8 * ((gpa >> sh) & 511));
        if (!(e & 7)) return r;
        r.code = DEVIRT_EPT_MISCONFIG;
        if ((e & 3) == 2) return r;
        perm &= e;
        const bool leaf = lvl == 1 || ((lvl == 3 || lvl == 2) && (e & 0x80));
        if (!leaf) {
            if (e & 0xF8) return r;
            table = e & kAddrMask;
            if (table >= arena_bytes || arena_bytes - table < 4096) return r;
            r.code = DEVIRT_EPT_VIOLATION;
            continue;
        }
        const uint64_t mt = (e >> 3) & 7;
        if (mt == 2 || mt == 3 || mt == 7) return r;
        const uint64_t low = (1ull << sh) - 1;
        if (e & low & ~0xFFFull) return r;
        const uint64_t h = (e & kAddrMask) | (gpa & low);
        const uint64_t pg = h & ~0xFFFull;
        if (pg >= arena_bytes || arena_bytes - pg < 4096) return r;
        r.code = DEVIRT_EPT_VIOLATION;
        if (need & ~perm & 3) return r;
        r.hpa = h;
        r.code = DEVIRT_OK;
        return r;
    }
    return r;
}

// GPA -> arena offset for an access that needs `need`: the memslots, or the
// EPT walk when the VM has one.
__device__ __forceinline__ uint32_t gpa_xlat(const DVm &v, uint64_t gpa, uint32_t need, uint64_t &hpa) {
    if (v.ept_root == kNoEpt) return slot_lookup(v, gpa, hpa) ? DEVIRT_OK : DEVIRT_NO_MEMSLOT;
    const XRes r = ept_walk(v.arena, v.arena_bytes, v.ept_root, gpa, need);
    if (r.code == DEVIRT_OK) hpa = r.hpa;
    return r.code;
}

// ------------------------------------------------------------ upper levels
// Result of walking the levels above the page directory for one 1 GiB region
// (x86-64: level 5 (LA57), level 4, level 3).
struct CEnt {
    uint64_t key;      // (asid << 27) | (gva >> 30); ~0 when empty
    uint64_t base;     // table: GPA of the level-2 table; 1 GiB leaf: frame GPA
    uint64_t path[3];  // arena offsets of the entries read, top level first
    uint32_t info;     // code:4 level:4 leaf1g:1 u:1 w:1 npath:2 abits:3 dbit:1
    uint32_t pad;
};
__device__ __forceinline__ uint32_t ci_code(uint32_t i) { return i & 15u; }
__device__ __forceinline__ uint32_t ci_level(uint32_t i) { return (i >> 4) & 15u; }
__device__ __forceinline__ uint32_t ci_leaf(uint32_t i) { return (i >> 8) & 1u; }
__device__ __forceinline__ uint32_t ci_u(uint32_t i) { return (i >> 9) & 1u; }
__device__ __forceinline__ uint32_t ci_w(uint32_t i) { return (i >> 10) & 1u; }
__device__ __forceinline__ uint32_t ci_np(uint32_t i) { return (i >> 11) & 3u; }
__device__ __forceinline__ uint32_t ci_abits(uint32_t i) { return (i >> 13) & 7u; }
constexpr uint32_t kCiDbit = 1u << 16;

template <int LEVELS>
__device__ __forceinline__ void walk_upper_t(const DVm &v, uint64_t cr3, uint64_t gva, CEnt &c) {
    uint64_t table = cr3 & kAddrMask;
    uint32_t u = 1, w = 1, abits = 0;
    c.path[0] = c.path[1] = c.path[2] = 0;
#pragma unroll
    for (int i = 0; i < LEVELS - 2; ++i) {
        const int lvl = LEVELS - i;
        const uint32_t shift = 12 + 9 * (lvl - 1);
        uint64_t th;
        const uint32_t xc = gpa_xlat(v, table, kNeedTable, th);
        if (xc) {
            c.info = xc | (lvl << 4) | (i << 11) | (abits << 13);
            return;
        }
        uint64_t eoff = th + 8 * ((gva >> shift) & 511);
        uint64_t e = load_entry(v.arena, eoff);
        c.path[i] = eoff;
        if (e & kA) abits |= 1u << i;
        if (!(e & kP)) {
            c.info = DEVIRT_NOT_PRESENT | (lvl << 4) | ((i + 1) << 11) | (abits << 13);
            return;
        }
        u &= (uint32_t)(e >> 2) & 1u;
        w &= (uint32_t)(e >> 1) & 1u;
        if (lvl >= 4 && (e & kPS)) {
            c.info = DEVIRT_RESERVED | (lvl << 4) | ((i + 1) << 11) | (abits << 13);
            return;
        }
        if (lvl == 3 && (e & kPS)) {
            if (e & 0x3FFFE000ull) {  // bits 29:13 of a 1 GiB leaf are reserved
                c.info = DEVIRT_RESERVED | (3u << 4) | ((i + 1) << 11) | (abits << 13);
                return;
            }
            c.base = e & kAddrMask & ~((1ull << 30) - 1);
            c.info = DEVIRT_OK | (1u << 8) | (u << 9) | (w << 10) | ((i + 1) << 11) | (abits << 13) |
                     ((e & kD) ? kCiDbit : 0u);
            return;
        }
        table = e & kAddrMask;
    }
    c.base = table;
    c.info = DEVIRT_OK | (u << 9) | (w << 10) | ((LEVELS - 2) << 11) | (abits << 13);
}

// PAE, the paper's 32-bit platform (section 6.2): one read of the 4-entry
// root table at CR3 bits 31:5, indexed by address bits 31:30.  Its entries
// grant every permission and take no accessed bit, so the cached path is
// empty; bits 2:1, 8:5 and 63:52 are reserved.
__device__ __forceinline__ void walk_upper_pae(const DVm &v, uint64_t cr3, uint64_t gva, CEnt &c) {
    c.path[0] = c.path[1] = c.path[2] = 0;
    uint64_t th;
    const uint32_t xc = gpa_xlat(v, cr3 & 0xFFFFFFE0ull, kNeedTable, th);
    if (xc) {
        c.info = xc | (3u << 4);
        return;
    }
    const uint64_t e = load_entry(v.arena, th + 8 * ((gva >> 30) & 3));
    if (!(e & kP)) {
        c.info = DEVIRT_NOT_PRESENT | (3u << 4);
        return;
    }
    if (e & kPaeRootRsvd) {
        c.info = DEVIRT_RESERVED | (3u << 4);
        return;
    }
    c.base = e & kAddrMask;
    c.info = DEVIRT_OK | (1u << 9) | (1u << 10);  // u = w = 1, no path entries
}

__device__ __forceinline__ void walk_upper(const DVm &v, uint64_t cr3, uint32_t levels, uint64_t gva, CEnt &c) {
    if (levels == 5)
        walk_upper_t<5>(v, cr3, gva, c);
    else if (levels == 3)
        walk_upper_pae(v, cr3, gva, c);
    else
        walk_upper_t<4>(v, cr3, gva, c);
}

__device__ __forceinline__ uint64_t user_limit(uint32_t levels) {
    return levels == 5 ? (1ull << 56) : levels == 3 ? (1ull << 32) : (1ull << 47);
}

__device__ __forceinline__ uint32_t cache_slot(uint64_t key) {
    uint64_t h = key ^ (key >> 7) ^ (key >> 17) ^ (key >> 29);
    return (uint32_t)h & (kCacheWays - 1);
}

// Look up (or fill) the 1 GiB-region cache for the calling lanes with
// `want` set.  Cross-lane safe: only the lane that wins a slot writes it.
// Must be called by the whole wavefront (uniform control flow).
__device__ __forceinline__ void cache_resolve(CEnt *cache, uint32_t *owner, bool want, uint64_t key,
                                              const DVm &v, uint64_t cr3, uint32_t levels, uint64_t gva, CEnt &c,
                                              uint32_t &slot, bool &hit) {
    const int lane = lane_id();
    hit = false;
    slot = cache_slot(key);
    if (want) {
        c = cache[slot];
        hit = (c.key == key);
        if (!hit) {
            walk_upper(v, cr3, levels, gva, c);
            c.key = key;
        }
    }
    bool miss = want && !hit;
    if (miss) owner[slot] = (uint32_t)lane;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (miss && owner[slot] == (uint32_t)lane) cache[slot] = c;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------- copying
// 16 output bytes from the 20-byte window (c.x c.y c.z c.w nx), starting at
// byte a (0..3); v_alignbyte takes the shift per lane.
__device__ __forceinline__ u32x4 funnel4(u32x4 c, uint32_t nx, uint32_t a) {
    u32x4 r;
    r.x = __builtin_amdgcn_alignbyte(c.y, c.x, a);
    r.y = __builtin_amdgcn_alignbyte(c.z, c.y, a);
    r.z = __builtin_amdgcn_alignbyte(c.w, c.z, a);
    r.w = __builtin_amdgcn_alignbyte(nx, c.w, a);
    return r;
}

__device__ __forceinline__ void store16(g_u32x4 *p, u32x4 v, bool nt) {
    if (nt)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// 16 bytes read at a 4-byte aligned address (one global_load_dwordx4).
typedef u32x4 u32x4_w4 __attribute__((aligned(4)));
typedef DV_GLOBAL u32x4_w4 g_u32x4_w4;

// Copy of n bytes by a group of G consecutive lanes of one wavefront; l is
// the lane's index in its group.  G = 64: the whole wavefront, arguments
// wave-uniform.  G = 16: each quarter of the wavefront copies its own
// segment, so a wavefront keeps four short segments in flight.
//
// The destination is written as aligned 16-byte blocks, with byte stores for
// the unaligned head and the tail (< 16 bytes each): no store touches a byte
// outside [dst, dst+n).  Block i takes its bytes from the 20-byte window at
// sa + 16 i, where sa is the 4-byte aligned address a bytes below the first
// body byte: the lane loads 16 bytes and takes the next dword from the next
// lane of its group (or, for the group's last lane, from the first lane of
// the next row).  Every load lies in an aligned dword that holds at least one
// source byte.  A pass moves 4 rows of G blocks and issues all of its loads
// before any store.
template <int G>
__device__ __forceinline__ void copy_span(uint8_t *dst_, const uint8_t *src_, uint32_t n, bool nt, int l) {
    constexpr int R = 4;
    if (n == 0) return;
    g_u8 *__restrict__ dst = gp<g_u8>(dst_);
    const g_u8 *__restrict__ src = gp<const g_u8>(src_);
    uint32_t h = (16u - (uint32_t)((uintptr_t)dst_ & 15u)) & 15u;
    if (h > n) h = n;
    const int32_t m = (int32_t)((n - h) >> 4);  // whole 16-byte destination blocks
    const uint32_t t = (n - h) & 15u;
    const uint32_t a = (uint32_t)((uintptr_t)(src_ + h) & 3u);
    const g_u8 *__restrict__ sa = src + h - a;
    g_u8 *__restrict__ db = dst + h;
    const uint32_t tail_off = h + 16u * (uint32_t)m;
    const int lane = lane_id();
    const int nb = (lane & ~(G - 1)) | ((lane + 1) & (G - 1));  // next lane of the group, cyclically
    int32_t b0 = 0;
    do {
        const bool first = b0 == 0;
        const bool last = b0 + R * G >= m;
        const int32_t rem = m - b0 - l;  // block b0 + l + G*u exists when G*u < rem
        const g_u8 *__restrict__ ps = sa + 16 * (int64_t)(b0 + l);
        g_u32x4 *pd = (g_u32x4 *)(db + 16 * (int64_t)(b0 + l));
        uint8_t hb = 0, tb = 0;
        if (first && (uint32_t)l < h) hb = src[l];
        if (last && (uint32_t)l < t) tb = src[tail_off + l];
        u32x4 cur[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            cur[u] = (u32x4){0u, 0u, 0u, 0u};
            if (G * u < rem)
                cur[u] = *(const g_u32x4_w4 *)(ps + 16 * G * u);
            else if (a != 0 && G * u == rem)  // block m: only its first dword is needed
                cur[u].x = *(const g_u32 *)(ps + 16 * G * u);
        }
        uint32_t ex = 0;  // first dword of block b0 + R*G, for the group's last lane
        if (a != 0 && l == G - 1 && R * G <= rem + G - 1) ex = *(const g_u32 *)(ps + 16 * (G * (R - 1) + 1));
        if (first && (uint32_t)l < h) dst[l] = hb;
        uint32_t rot[R];
#pragma unroll
        for (int u = 0; u < R; ++u) rot[u] = (uint32_t)__shfl((int)cur[u].x, nb);
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const uint32_t nx = (l == G - 1) ? (u + 1 < R ? rot[u + 1 < R ? u + 1 : 0] : ex) : rot[u];
            if (G * u < rem) store16(pd + G * u, funnel4(cur[u], nx, a), nt);
        }
        if (last && (uint32_t)l < t) dst[tail_off + l] = tb;
        b0 += R * G;
    } while (b0 < m);
}

// Whole-wavefront copy (all arguments wave-uniform).
__device__ __forceinline__ void copy_wave(uint8_t *dst, const uint8_t *src, uint32_t n, bool nt) {
    copy_span<64>(dst, src, n, nt, lane_id());
}

// Copy by one lane (short segments).
__device__ __forceinline__ void copy_lane(uint8_t *dst_, const uint8_t *src_, uint32_t n) {
    g_u8 *dst = gp<g_u8>(dst_);
    const g_u8 *src = gp<const g_u8>(src_);
    for (uint32_t i = 0; i < n; ++i) dst[i] = src[i];
}

// ------------------------------------------------------ translate a group
// One wavefront, requests [r0, r0+gn) (or one request passed by value).
// Must be entered by all 64 lanes.
struct GroupOut {
    unsigned long long pages, hits, misses, segs, inl, atomics, spills;
};

// Requests of more than B.large_pages pages ("large"): in the batched path a
// group leaves them to k_translate_large, where the wavefronts of a workgroup
// walk one large request together.
enum : uint32_t {
    kLargeKeep = 0,   // walk them here
    kLargeDefer = 1,  // put them on the epoch's large list; their results come later
    kLargeSkip = 2,   // leave them alone (spill pass: a large request spills on its own)
};

// Workgroup-shared state of a large request walked by several wavefronts.
struct CoopShared {
    uint32_t ff[3];   // per round, rotating: the request's first faulting page (kNone: none)
    uint32_t fcode, flevel;
    uint64_t flo;     // that page's first byte in the request
    uint32_t queued;  // segments queued
    uint32_t spilled;
};

// Returns (wave-uniformly) true when some run of the group found its queue
// part full while B.spill_mode is set: such runs are neither queued nor
// copied, and the caller puts the group on the epoch's spill list.
//
// kCoop: the wavefronts of a workgroup walk one large request (gn = 1)
// together, round by round: in each round wavefront w takes pages
// [64 w, 64 w + 64) of the round's 64 W.  The walk of a round has no side
// effects; the request's first faulting page is then agreed in LDS (cs), and
// only pages before it get A/D bits and copies, as in the one-wavefront walk.
// All wavefronts run the same rounds (barriers inside); the result is written
// by wavefront 0.  e0: the epoch's first request (slot of the large list).
template <bool kPlain, bool kCoop>
__device__ bool process_group(const DView &V, const DBatch &B, uint64_t r0, uint32_t gn,
                              const devirt_request &preq, uint32_t epoch, CEnt *cache, uint32_t *owner,
                              bool coop_all, uint32_t large_mode, uint64_t e0, DEpochCtr *ctr, GroupOut &st,
                              CoopShared *cs) {
    const int lane = lane_id();
    const uint32_t nw = kCoop ? (blockDim.x >> 6) : 1u;    // wavefronts walking the request
    const uint32_t wv = kCoop ? (threadIdx.x >> 6) : 0u;   // this one
    // this wavefront's part of the segment queues
    const uint32_t qpart = kPlain ? 0u : (uint32_t)((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % kQParts);
    const uint64_t pcap = B.part_cap;
    // ---- load and validate the group's requests (lane k owns request k)
    uint64_t gva = 0, host = 0, cr3 = 0;
    uint32_t len = 0, asid = 0, dir = 0, vm = 0, levels = 4, code0 = 0, nch = 0;
    if ((uint32_t)lane < gn) {
        devirt_request rq;
        if (kPlain) {
            rq = preq;
        } else {
            const g_u32x4 *p = gp<const g_u32x4>(B.reqs + r0 + lane);
            u32x4 a = p[0], b = p[1];
            rq.gva = ((uint64_t)a.y << 32) | a.x;
            rq.host = ((uint64_t)a.w << 32) | a.z;
            rq.len = b.x;
            rq.asid = b.y;
            rq.dir = (uint8_t)(b.z & 0xFF);
        }
        gva = rq.gva;
        host = rq.host;
        len = rq.len;
        asid = rq.asid;
        dir = rq.dir ? 1u : 0u;
        if (asid >= V.nproc) {
            code0 = DEVIRT_INVALID;
        } else {
            DProc p = gp<const DV_GLOBAL DProc>(V.procs)[asid];
            vm = p.vm;
            levels = p.levels;
            cr3 = p.cr3;
            if (len != 0) {
                uint64_t lim = user_limit(levels);
                if (gva >= lim || (uint64_t)len > lim - gva)
                    code0 = DEVIRT_NONCANONICAL;
                else
                    nch = (uint32_t)(((gva + len - 1) >> 12) - (gva >> 12) + 1);
            }
        }
    }
    // large requests left to k_translate_large (or to their own spill entry)
    bool large = false;
    if (!kPlain && !kCoop && large_mode != kLargeKeep && B.large_pages && nch > B.large_pages) {
        large = true;
        nch = 0;
    }
    if (!kPlain && !kCoop && large_mode == kLargeDefer) {
        const uint64_t lm = __ballot(large);
        if (lm) {
            uint32_t lb = 0;
            if (lane == 0) lb = atomicAdd(&ctr[epoch].large_n, (uint32_t)__popcll(lm));
            lb = shfl32(lb, 0);
            if (large) gp<g_u64>(B.large)[e0 + lb + (uint32_t)__popcll(lm & mask_lt(lane))] = r0 + (uint64_t)lane;
        }
    }
    // ---- wave exclusive prefix sum of page counts
    uint32_t incl = nch;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = shfl32(incl, lane >= d ? lane - d : lane);
        if (lane >= d) incl += t;
    }
    const uint32_t start = incl - nch;
    const uint32_t total = shfl32(incl, 63);

    // ---- per-request path: the process's translation cache, a FIFO whose
    // slots live in lanes 0..cap-1 (section 4.2).  A page held in it (and,
    // for a write into the guest, held from a write) is not walked: its
    // translation comes from the slot, and the bits a walk would set are
    // already set.  Lookups are replayed in page order after each pass, so
    // hits, misses and evictions are those of a sequential FIFO.
    const uint32_t cap = B.fifo_entries;
    const bool use_fifo = kPlain && B.fifo != nullptr && cap != 0 && total > 0;
    DFifo *fifo = nullptr;
    uint64_t fv = ~0ull, fh = 0;
    uint32_t f_occ = 0, f_wr = 0, f_n = 0, f_head = 0;
    unsigned long long f_hits = 0, f_miss = 0;
    if (use_fifo) {
        fifo = B.fifo + uniform_u32(asid);  // kPlain: lane 0 holds the request
        if (uniform_u64(*gp<const g_u64>(&fifo->gen)) == B.xlat_gen) {
            f_n = uniform_u32(*gp<const g_u32>(&fifo->n));
            f_head = uniform_u32(*gp<const g_u32>(&fifo->head));
            f_wr = uniform_u32(*gp<const g_u32>(&fifo->written));
            if ((uint32_t)lane < cap) {
                fv = gp<const g_u64>(fifo->vpn)[lane];
                fh = gp<const g_u64>(fifo->hpa)[lane];
            }
            for (uint32_t k = 0; k < f_n; ++k) f_occ |= 1u << ((f_head + k) % cap);
        }
    }

    // per-request (owner lane) state
    uint32_t ff = kNone, fcode = 0, flevel = 0, queued = 0;
    uint64_t flo = 0;
    bool spilled = false;

    // kCoop: round r is walked by min(nw, 2^r) wavefronts, so that a request
    // faulting early is walked little past its fault (as by one wavefront),
    // and one that keeps going soon has every wavefront on it
    uint32_t round = 0, nr = 1;
    for (uint32_t rb = 0; rb < total; rb += 64 * nr, ++round) {
        nr = kCoop ? (round < 5 && (1u << round) < nw ? (1u << round) : nw) : 1u;  // wavefronts this round
        const uint32_t base = rb + 64 * wv;
        const uint32_t c = base + (uint32_t)lane;
        const bool active = wv < nr && c < total;
        // owner of page c: the last request whose start <= c
        int j = 0;
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) {
            int cand = j + s;
            int idx = cand < (int)gn ? cand : (int)gn - 1;
            uint32_t sj = shfl32(start, idx);
            if (cand < (int)gn && sj <= c) j = cand;
        }
        const uint64_t j_gva = shfl64(gva, j);
        const uint64_t j_host = shfl64(host, j);
        const uint64_t j_cr3 = shfl64(cr3, j);
        const uint32_t j_len = shfl32(len, j);
        const uint32_t j_meta = shfl32(dir | (levels << 1) | (vm << 4), j);
        const uint32_t j_asid = shfl32(asid, j);
        const uint32_t j_start = shfl32(start, j);
        const uint32_t j_ff = kCoop ? kNone : shfl32(ff, j);  // kCoop: rounds end at the first fault
        const uint32_t j_dir = j_meta & 1u, j_levels = (j_meta >> 1) & 7u, j_vm = j_meta >> 4;
        const bool work = active && j_ff == kNone;

        const uint32_t k = c - j_start;  // page index inside the request
        const uint64_t page = (j_gva & ~0xFFFull) + ((uint64_t)k << 12);
        const uint64_t lo = page > j_gva ? page : j_gva;
        const uint64_t end = j_gva + j_len;
        const uint64_t hi = page + 4096 < end ? page + 4096 : end;

        // pages the translation cache holds (as of the start of this pass) skip the walk
        bool fhit = false;
        uint64_t fhpa = 0;
        if (use_fifo) {
            for (uint32_t e = 0; e < cap; ++e) {
                const uint64_t ve = uniform_u64(shfl64(fv, (int)e));
                const uint64_t he = uniform_u64(shfl64(fh, (int)e));
                if (work && ((f_occ >> e) & 1u) && ve == (lo >> 12) && (!j_dir || ((f_wr >> e) & 1u))) {
                    fhit = true;
                    fhpa = he;
                }
            }
        }
        const bool walkl = work && !fhit;

        // ---- heads: first lane of each (request, 2 MiB region) run of walking lanes
        const int prev = lane > 0 ? lane - 1 : 0;
        const uint32_t p_work = shfl32(walkl ? 1u : 0u, prev);
        const uint32_t p_j = shfl32((uint32_t)j, prev);
        const uint64_t p_lo = shfl64(lo, prev);
        const bool head = walkl && (lane == 0 || !p_work || p_j != (uint32_t)j || (p_lo >> 21) != (lo >> 21));
        const uint64_t head_mask = __ballot(head);

        DVm vmv;
        if (work) vmv = load_vm(V, j_vm, V.lds != 0);
        // upper levels through the cache (heads only)
        CEnt ce;
        ce.info = 0;
        ce.base = 0;
        ce.path[0] = ce.path[1] = ce.path[2] = 0;
        uint32_t cslot;
        bool chit;
        const uint64_t key1 = ((uint64_t)j_asid << 27) | (lo >> 30);
        cache_resolve(cache, owner, head, key1, vmv, j_cr3, j_levels, lo, ce, cslot, chit);
        if (head) {
            if (chit)
                st.hits++;
            else
                st.misses++;
        }
        // level 2 (heads): rkind 0 = 4 KiB table, 1 = 2 MiB leaf, 2 = 1 GiB leaf
        uint32_t rcode = 0, rlevel = 0, rkind = 0, ru = 0, rw = 0, rhas = 0;
        uint64_t rbase = 0, pde_off = 0;
        if (head) {
            rcode = ci_code(ce.info);
            rlevel = ci_level(ce.info);
            ru = ci_u(ce.info);
            rw = ci_w(ce.info);
            if (rcode == 0) {
                if (ci_leaf(ce.info)) {
                    rkind = 2;
                    rbase = ce.base;
                } else {
                    uint64_t th;
                    const uint32_t xc = gpa_xlat(vmv, ce.base, kNeedTable, th);
                    if (xc) {
                        rcode = xc;
                        rlevel = 2;
                    } else {
                        pde_off = th + 8 * ((lo >> 21) & 511);
                        uint64_t e = load_entry(vmv.arena, pde_off);
                        rhas = (e & kA) ? 1u : 0u;
                        if (e & kD) rhas |= 2u;
                        if (!(e & kP)) {
                            rcode = DEVIRT_NOT_PRESENT;
                            rlevel = 2;
                        } else if (j_levels == 3 && (e & kPaeRsvd)) {
                            rcode = DEVIRT_RESERVED;
                            rlevel = 2;
                        } else {
                            ru &= (uint32_t)(e >> 2) & 1u;
                            rw &= (uint32_t)(e >> 1) & 1u;
                            if (e & kPS) {
                                if (e & 0x1FE000ull) {  // bits 20:13 of a 2 MiB leaf are reserved
                                    rcode = DEVIRT_RESERVED;
                                    rlevel = 2;
                                } else {
                                    rkind = 1;
                                    rbase = e & kAddrMask & ~((1ull << 21) - 1);
                                }
                            } else {
                                uint64_t pt;
                                const uint32_t xc1 = gpa_xlat(vmv, e & kAddrMask, kNeedTable, pt);
                                if (xc1) {
                                    rcode = xc1;
                                    rlevel = 1;
                                } else {
                                    rkind = 0;
                                    rbase = pt;
                                }
                            }
                        }
                    }
                }
            }
        }
        // ---- broadcast the region result from each head to its lanes
        const int h = 63 - __clzll(head_mask & mask_le(lane));
        const int hsrc = (head_mask & mask_le(lane)) ? h : lane;
        const uint32_t r_packed =
            shfl32(rcode | (rlevel << 4) | (rkind << 8) | (ru << 10) | (rw << 11) | (rhas << 12), hsrc);
        const uint64_t r_base = shfl64(rbase, hsrc);

        // ---- leaf step (every walking lane)
        uint32_t code = 0, level = 0, shift = 0;
        uint64_t gpa = 0, hpa = 0, leaf_off = 0, leaf_e = 0;
        if (fhit) hpa = fhpa + (lo & 0xFFFull);
        if (walkl) {
            code = r_packed & 15u;
            level = (r_packed >> 4) & 15u;
            const uint32_t kind = (r_packed >> 8) & 3u;
            uint32_t u = (r_packed >> 10) & 1u, w = (r_packed >> 11) & 1u;
            uint32_t leaf_level = 0;
            uint64_t frame = 0;
            if (code == 0) {
                if (kind == 0) {
                    leaf_off = r_base + 8 * ((lo >> 12) & 511);
                    leaf_e = load_entry(vmv.arena, leaf_off);
                    if (!(leaf_e & kP)) {
                        code = DEVIRT_NOT_PRESENT;
                        level = 1;
                    } else if (j_levels == 3 && (leaf_e & kPaeRsvd)) {
                        code = DEVIRT_RESERVED;
                        level = 1;
                    } else {
                        u &= (uint32_t)(leaf_e >> 2) & 1u;
                        w &= (uint32_t)(leaf_e >> 1) & 1u;
                        frame = leaf_e & kAddrMask;
                        shift = 12;
                        leaf_level = 1;
                    }
                } else {
                    frame = r_base;
                    shift = kind == 1 ? 21 : 30;
                    leaf_level = kind == 1 ? 2 : 3;
                }
            }
            if (code == 0) {
                gpa = frame | (lo & ((1ull << shift) - 1));
                if (!u) {
                    code = DEVIRT_PROT_USER;
                    level = leaf_level;
                } else if (j_dir && !w) {
                    code = DEVIRT_PROT_WRITE;
                    level = leaf_level;
                } else {
                    const uint32_t xc = gpa_xlat(vmv, gpa, j_dir ? kNeedW : kNeedR, hpa);
                    if (xc) {
                        code = xc;
                        level = 0;
                    }
                }
            }
        }
        st.pages += __popcll(__ballot(work));

        // ---- first fault per request, pages that will be copied
        const uint64_t fmask = __ballot(work && code != 0);
        const uint32_t jfirst = j_start > base ? j_start - base : 0u;  // first lane of request j
        const uint64_t jmask = mask_le(lane) & ~mask_lt((int)jfirst);
        uint32_t ffr = kNone;  // kCoop: the request's first faulting page, agreed by the workgroup
        if (kCoop) {
            if (lane == 0 && fmask)
                atomicMin(&cs->ff[round % 3], base + (uint32_t)(__ffsll((unsigned long long)fmask) - 1));
            __syncthreads();
            ffr = uniform_u32(*(volatile uint32_t *)&cs->ff[round % 3]);
            if (threadIdx.x == 0) cs->ff[(round + 2) % 3] = kNone;  // every wave is done reading it
            if (work && c == ffr) {
                cs->fcode = code;
                cs->flevel = level;
                cs->flo = lo;
            }
        }
        const bool copied = kCoop ? (work && code == 0 && c < ffr) : (work && code == 0 && (fmask & jmask) == 0);
        // (pages served by the translation cache need no A/D: their filling walk set them)
        const uint64_t cmask = __ballot(copied && !fhit);
        const uint64_t cto_mask = __ballot(copied && !fhit && j_dir);

        // owner lanes pick up their request's first fault in this pass
        if (!kCoop) {
            const bool own = (uint32_t)lane < gn && nch > 0 && ff == kNone;
            uint64_t my = 0;
            if (own) {
                uint32_t a = start > base ? start - base : 0u;
                uint32_t b = start + nch - base;  // may exceed 64
                if (start < base + 64 && start + nch > base) {
                    uint64_t hi_m = b >= 64 ? ~0ull : ((1ull << b) - 1);
                    my = fmask & hi_m & ~mask_lt((int)a);
                }
            }
            const int f = my ? (__ffsll((unsigned long long)my) - 1) : lane;
            const uint32_t f_code = shfl32(code, f);
            const uint32_t f_level = shfl32(level, f);
            const uint64_t f_lo = shfl64(lo, f);
            if (own && my) {
                ff = base + (uint32_t)f - start;
                fcode = f_code;
                flevel = f_level;
                flo = f_lo;
            }
        }

        // ---- translation cache: this pass's lookups in page order, up to and
        // including the request's first faulting page (kPlain: one request)
        if (use_fifo) {
            uint64_t lk = __ballot(work);
            if (fmask) lk &= mask_le(__ffsll((unsigned long long)fmask) - 1);
            const uint64_t okm = __ballot(work && code == 0);
            const uint64_t pg = hpa - (lo & 0xFFFull);  // the page's arena offset (lanes that translated)
            while (lk) {
                const int jl = __ffsll((unsigned long long)lk) - 1;
                lk &= lk - 1;
                const uint64_t v = uniform_u64(shfl64(lo >> 12, jl));
                const uint64_t hp = uniform_u64(shfl64(pg, jl));
                const bool wrj = uniform_u32(shfl32(j_dir, jl)) != 0;
                const uint64_t em = __ballot((uint32_t)lane < cap && ((f_occ >> lane) & 1u) && fv == v);
                const int slot = em ? __ffsll((unsigned long long)em) - 1 : -1;
                if (slot >= 0 && (!wrj || ((f_wr >> slot) & 1u))) {
                    f_hits++;
                    continue;
                }
                f_miss++;
                if (!((okm >> jl) & 1ull)) continue;  // a failed walk inserts nothing
                if (slot >= 0) {                      // held from reads: now written
                    f_wr |= 1u << slot;
                    continue;
                }
                uint32_t tail;
                if (f_n == cap) {  // full: the oldest entry leaves
                    tail = f_head;
                    f_head = (f_head + 1) % cap;
                } else {
                    tail = (f_head + f_n) % cap;
                    f_n++;
                }
                if ((uint32_t)lane == tail) {
                    fv = v;
                    fh = hp;
                }
                f_occ |= 1u << tail;
                f_wr = (f_wr & ~(1u << tail)) | ((wrj ? 1u : 0u) << tail);
            }
        }

        // ---- A/D: leaf of 4 KiB pages per lane; region-level entries by heads
        uint32_t atomics = 0;
        if (copied && leaf_off) {
            const uint32_t want = (uint32_t)kA | (j_dir ? (uint32_t)kD : 0u);
            if (((uint32_t)leaf_e & want) != want) {
                or_entry(vmv.arena, leaf_off, want);
                atomics++;
            }
        }
        if (head) {
            const int nh_bit = __ffsll((unsigned long long)(head_mask & ~mask_le(lane)));
            const int nh = nh_bit ? nh_bit - 1 : 64;
            const uint64_t rmask = mask_lt(nh) & ~mask_lt(lane);
            if (cmask & rmask) {
                const bool rto = (cto_mask & rmask) != 0;
                // level-2 entry (a table pointer or a 2 MiB leaf)
                if (rkind == 0 || rkind == 1) {
                    uint32_t want = (uint32_t)kA | ((rkind == 1 && rto) ? (uint32_t)kD : 0u);
                    if ((rhas & want) != want) {
                        or_entry(vmv.arena, pde_off, want);
                        atomics++;
                    }
                }
                // levels 5..3 from the cached walk
                const uint32_t np = ci_np(ce.info), ab = ci_abits(ce.info);
                uint32_t mark = 0;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    if ((uint32_t)i < np) {
                        uint32_t want = (uint32_t)kA;
                        const bool is_leaf = rkind == 2 && (uint32_t)i + 1 == np;
                        bool need = !((ab >> i) & 1u);
                        if (is_leaf && rto) {
                            want |= (uint32_t)kD;
                            need = need || !(ce.info & kCiDbit);
                        }
                        if (need) {
                            or_entry(vmv.arena, ce.path[i], want);
                            atomics++;
                        }
                        mark |= 1u << (13 + i);
                        if (is_leaf && rto) mark |= kCiDbit;
                    }
                }
                if (cache[cslot].key == key1) atomicOr(&cache[cslot].info, mark);
            }
        }
        st.atomics += atomics;

        // ---- copy segments: runs of pages whose guest side is contiguous
        uint8_t *const arena = work ? vmv.arena : nullptr;
        const uint64_t gptr = (uint64_t)(uintptr_t)arena + hpa;
        const uint64_t hptr = j_host + (lo - j_gva);
        const uint32_t nbytes = (uint32_t)(hi - lo);
        const uint32_t p_copied = shfl32(copied ? 1u : 0u, prev);
        const uint64_t p_gptr = shfl64(gptr, prev);
        const uint32_t p_n = shfl32(nbytes, prev);
        const bool cont = copied && lane > 0 && p_copied && p_j == (uint32_t)j && p_gptr + p_n == gptr &&
                          (k % B.seg_chunks) != 0;
        const bool rhead = copied && !cont;
        const uint64_t cont_mask = __ballot(cont);
        // run [lane, e): e = first later lane that does not continue the run
        const int e_bit = __ffsll((unsigned long long)(~cont_mask & ~mask_le(lane)));
        const int e = e_bit ? e_bit - 1 : 64;
        const int last = rhead ? e - 1 : lane;
        const uint64_t l_end = shfl64(lo + nbytes, last);
        const uint32_t run = rhead ? (uint32_t)(l_end - lo) : 0u;
        uint64_t src = 0, dst = 0;
        if (rhead) {
            src = j_dir ? hptr : gptr;
            dst = j_dir ? gptr : hptr;
        }
        const bool small = rhead && !coop_all && run <= B.inline_bytes;
        if (small) copy_lane((uint8_t *)dst, (const uint8_t *)src, run);
        const bool want_q = rhead && !small && !coop_all;
        const bool is_short = run <= kShortRun;
        const uint64_t lmask = __ballot(want_q && !is_short);
        const uint64_t smask = __ballot(want_q && is_short);
        bool coop = rhead && coop_all;
        uint32_t q_ok = 0;
        if (lmask | smask) {
            uint32_t lbase = 0, sbase = 0;
            if (lane == 0) {
                if (lmask) lbase = atomicAdd(&ctr[epoch].q[qpart][0], (uint32_t)__popcll(lmask));
                if (smask) sbase = atomicAdd(&ctr[epoch].q[kQParts + qpart][0], (uint32_t)__popcll(smask));
            }
            lbase = shfl32(lbase, 0);
            sbase = shfl32(sbase, 0);
            if (want_q) {
                const uint64_t qm = is_short ? smask : lmask;
                const uint64_t pos = (uint64_t)(is_short ? sbase : lbase) + (uint64_t)__popcll(qm & mask_lt(lane));
                if (pos < pcap) {
                    DSeg sg;
                    sg.src = src;
                    sg.dst = dst;
                    sg.len = run;
                    sg.req = (uint32_t)(r0 + (uint64_t)j);
                    sg.pad = 0;
                    gp<DV_GLOBAL DSeg>(is_short ? B.shorts : B.segs)[qpart * pcap + pos] = sg;
                    q_ok = 1;
                } else if (B.spill_mode) {
                    spilled = true;  // queue full: the spill pass copies it
                } else {
                    coop = true;  // queue full: the wavefront copies it below
                }
            }
        }
        st.segs += __popcll(__ballot(q_ok != 0));
        st.inl += __popcll(__ballot(small || coop));  // inline and queue-overflow copies
        // per-request count of queued segments (for completion times)
        {
            const uint64_t okm = __ballot(q_ok != 0);
            if ((uint32_t)lane < gn && nch > 0 && start < base + 64 && start + nch > base) {
                uint32_t a = start > base ? start - base : 0u;
                uint32_t b = start + nch - base;
                uint64_t hi_m = b >= 64 ? ~0ull : ((1ull << b) - 1);
                queued += (uint32_t)__popcll(okm & hi_m & ~mask_lt((int)a));
            }
        }
        uint64_t cm = __ballot(coop);
        while (cm) {
            const int l = __ffsll((unsigned long long)cm) - 1;
            const uint64_t s = uniform_u64(shfl64(src, l)), d = uniform_u64(shfl64(dst, l));
            const uint32_t n = uniform_u32(shfl32(run, l));
            copy_wave((uint8_t *)d, (const uint8_t *)s, n, B.nontemporal != 0);
            cm &= cm - 1;
        }
        if (kCoop && ffr != kNone) {  // workgroup-uniform
            ff = ffr;
            break;
        }
    }
    bool any_spill = __ballot(spilled) != 0;
    if (kCoop) {
        // the request's outcome, from the workgroup's shared state
        if (lane == 0) {
            if (queued) atomicAdd(&cs->queued, queued);
            if (any_spill) atomicOr(&cs->spilled, 1u);
        }
        __syncthreads();
        any_spill = *(volatile uint32_t *)&cs->spilled != 0;
        queued = *(volatile uint32_t *)&cs->queued;
        if (ff != kNone) {
            fcode = *(volatile uint32_t *)&cs->fcode;
            flevel = *(volatile uint32_t *)&cs->flevel;
            flo = *(volatile uint64_t *)&cs->flo;
        }
    }

    // ---- results (owner lanes; a large request's come from k_translate_large)
    if ((uint32_t)lane < gn && !large && wv == 0) {
        devirt_result r;
        r.pad = 0;
        if (code0) {
            r.bytes_done = 0;
            r.fault_gva = gva;
            r.code = code0;
            r.level = 0;
        } else if (ff == kNone) {
            r.bytes_done = len;
            r.fault_gva = 0;
            r.code = 0;
            r.level = 0;
        } else {
            r.bytes_done = flo - gva;
            r.fault_gva = flo;
            r.code = fcode;
            r.level = (uint16_t)flevel;
        }
        gp<DV_GLOBAL devirt_result>(B.res)[kPlain ? 0 : r0 + lane] = r;
        if (!kPlain && B.t_done) {
            B.pending[r0 + lane] = queued;
            if (queued == 0) B.t_done[r0 + lane] = now_ns(B);
        }
    }
    if (use_fifo) {
        if ((uint32_t)lane < cap) {
            gp<g_u64>(fifo->vpn)[lane] = fv;
            gp<g_u64>(fifo->hpa)[lane] = fh;
        }
        if (lane == 0) {
            *gp<g_u32>(&fifo->written) = f_wr;
            *gp<g_u32>(&fifo->n) = f_n;
            *gp<g_u32>(&fifo->head) = f_head;
            *gp<g_u64>(&fifo->gen) = B.xlat_gen;
            *gp<DV_GLOBAL unsigned long long>(&fifo->hits) += f_hits;
            *gp<DV_GLOBAL unsigned long long>(&fifo->misses) += f_miss;
        }
    }
    return any_spill;
}

// ------------------------------------------------------------------ kernels
__global__ void k_reset(DBatch b, uint32_t n_epochs) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *b.t0 = wall_clock64();
    constexpr uint32_t per = 3 + 2 * kQParts;  // counters per epoch
    for (; i < n_epochs * per; i += gridDim.x * blockDim.x) {
        const uint32_t e = i / per, k = i % per;
        if (k == 0)
            b.ctr[e].group_cursor = 0;
        else if (k == per - 2)
            b.ctr[e].spill_n = 0;
        else if (k == per - 1)
            b.ctr[e].large_n = 0;
        else
            b.ctr[e].q[k - 1][0] = 0;
    }
}

__device__ __forceinline__ void flush_counters(DCounters *c, const GroupOut &st) {
    if (!c) return;
    unsigned long long v[7] = {st.pages, st.hits, st.misses, st.segs, st.inl, st.atomics, st.spills};
    // lane-local partial sums -> one atomic per counter per wavefront
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        unsigned long long x = v[i];
        for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
        v[i] = x;
    }
    if (lane_id() == 0) {
        atomicAdd(&c->pages_walked, v[0] / 64);
        atomicAdd(&c->cache_hits, v[1]);
        atomicAdd(&c->cache_misses, v[2]);
        atomicAdd(&c->segments, v[3] / 64);
        atomicAdd(&c->inline_segments, v[4] / 64);
        atomicAdd(&c->ad_atomics, v[5]);
        atomicAdd(&c->spilled_groups, v[6] / 64);
    }
}

// direct != 0: the translating wavefronts copy their runs themselves and
// nothing is queued (one launch for a small batch).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_translate_groups(DView v, DBatch b, uint64_t r0, uint64_t r1, uint32_t epoch, int direct) {
    extern __shared__ uint8_t smem[];
    v.lds = lds_slots_load(v) ? 1u : 0u;
    const int wave = threadIdx.x >> 6;
    CEnt *cache = (CEnt *)smem + wave * kCacheWays;
    uint32_t *owner = (uint32_t *)((CEnt *)smem + (blockDim.x >> 6) * kCacheWays) + wave * kCacheWays;
    if ((threadIdx.x & 63) < kCacheWays) cache[threadIdx.x & 63].key = ~0ull;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const uint64_t n = r1 - r0;
    const uint32_t G = b.group;
    const uint64_t ngroups = (n + G - 1) / G;
    GroupOut st = {0, 0, 0, 0, 0, 0, 0};
    devirt_request dummy = {};
    // Each wavefront takes group (its global index) first, without an atomic;
    // further groups come from the cursor, numbered after those first ones.
    // The next claim is issued before the current group is translated, so its
    // round trip overlaps the group's own loads.  When every group is some
    // wavefront's first, no claim is made at all (and the cursor is not read).
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const bool claim = ngroups > nwaves;
    uint64_t gi = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (uint64_t)wave;
    while (gi < ngroups) {
        uint32_t g = 0;
        if (claim && lane_id() == 0) g = atomicAdd(&b.ctr[epoch].group_cursor, 1u);
        const uint64_t gs = r0 + gi * G;
        const uint32_t gn = (uint32_t)((r1 - gs) < G ? (r1 - gs) : G);
        if (process_group<false, false>(v, b, gs, gn, dummy, epoch, cache, owner, direct != 0,
                                        direct ? kLargeKeep : kLargeDefer, r0, b.ctr, st, nullptr)) {
            st.spills++;
            if (lane_id() == 0) {
                const uint32_t k = atomicAdd(&b.ctr[epoch].spill_n, 1u);
                gp<g_u64>(b.spill)[r0 + k] = gs;  // at most one slot per group of [r0, r1)
            }
        }
        if (!claim) break;
        gi = nwaves + uniform_u32(shfl32(g, 0));
    }
    flush_counters(b.counters, st);
}

// The epoch's large requests (listed by k_translate_groups), one per
// workgroup at a time: its wavefronts walk the request's pages together (see
// process_group), so a request of thousands of pages takes a few rounds
// instead of one wavefront's many passes.  Queue overflow is handled as in
// k_translate_groups; a request that spills goes on the spill list alone.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_translate_large(DView v, DBatch b, uint64_t r0, uint32_t epoch) {
    extern __shared__ uint8_t smem[];
    __shared__ CoopShared cs;
    const int wave = threadIdx.x >> 6;
    CEnt *cache = (CEnt *)smem + wave * kCacheWays;
    uint32_t *owner = (uint32_t *)((CEnt *)smem + (blockDim.x >> 6) * kCacheWays) + wave * kCacheWays;
    const uint32_t n = uniform_u32(*gp<const g_u32>(&b.ctr[epoch].large_n));
    if (n == 0) return;
    v.lds = lds_slots_load(v) ? 1u : 0u;
    if ((threadIdx.x & 63) < kCacheWays) cache[threadIdx.x & 63].key = ~0ull;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    GroupOut st = {0, 0, 0, 0, 0, 0, 0};
    devirt_request dummy = {};
    for (uint32_t k = blockIdx.x; k < n; k += gridDim.x) {
        const uint64_t r = uniform_u64(gp<const g_u64>(b.large)[r0 + k]);
        if (threadIdx.x == 0) {
            cs.ff[0] = cs.ff[1] = cs.ff[2] = kNone;
            cs.queued = 0;
            cs.spilled = 0;
        }
        __syncthreads();
        const bool sp = process_group<false, true>(v, b, r, 1, dummy, epoch, cache, owner, false, kLargeKeep, r0,
                                                   b.ctr, st, &cs);
        if (b.counters && threadIdx.x == 0) atomicAdd(&b.counters->large_requests, 1ull);
        if (sp && threadIdx.x == 0) {
            st.spills++;
            const uint32_t i = atomicAdd(&b.ctr[epoch].spill_n, 1u);
            gp<g_u64>(b.spill)[r0 + i] = r | kSpillOne;
        }
        __syncthreads();  // cs is reused for the next request
    }
    flush_counters(b.counters, st);
}

// Copy of one epoch's queued segments.  The copy is bound by the bytes it
// keeps in flight: hence at most 64 VGPRs, so that 8 wavefronts (the most a
// SIMD holds) stay resident, and short segments a 16-lane quarter each, so
// that a wavefront keeps up to four of them in flight.
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) k_copy(DBatch b, uint32_t epoch) {
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t w0 = uniform_u64((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    const bool nt = b.nontemporal != 0;
    const int lane = lane_id();
    const uint64_t pcap = b.part_cap;
    // lane p < 32: part p of the long queue; lane 32 + p: part p of the short
    // queue.  Exclusive scan of the part counts within each half.
    uint32_t cnt = b.ctr[epoch].q[lane][0];
    if (cnt > pcap) cnt = (uint32_t)pcap;
    uint32_t incl = cnt;
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
        const uint32_t t = shfl32(incl, (lane & 31) >= d ? lane - d : lane);
        if ((lane & 31) >= d) incl += t;
    }
    const uint32_t excl = incl - cnt;
    const uint32_t nlong = uniform_u32(shfl32(incl, 31));
    const uint32_t nshort = uniform_u32(shfl32(incl, 63));
    const bool lo_half = lane < 32;
    // queue index s lies in the last part whose exclusive start is <= s
    // (parts are in lane order, so those lanes form a prefix of the half)

    // long segments: one per wavefront
    const DV_GLOBAL DSeg *segs = gp<const DV_GLOBAL DSeg>(b.segs);
    for (uint64_t s = w0; s < nlong; s += waves) {
        const int p = 63 - __clzll(__ballot(lo_half && excl <= (uint32_t)s));
        const uint64_t i = (uint64_t)p * pcap + (s - (uint32_t)__builtin_amdgcn_readlane((int)excl, p));
        const DSeg sg = segs[i];
        copy_wave((uint8_t *)uniform_u64(sg.dst), (const uint8_t *)uniform_u64(sg.src), uniform_u32(sg.len), nt);
        if (b.t_done && lane == 0) {
            uint32_t old = atomicSub(&b.pending[sg.req], 1u);
            if (old == 1) b.t_done[sg.req] = now_ns(b);
        }
    }
    // short segments: one per 16-lane quarter, four per wavefront per round
    const DV_GLOBAL DSeg *sh = gp<const DV_GLOBAL DSeg>(b.shorts);
    const int q = lane >> 4, l = lane & 15;
    for (uint64_t s0 = 4 * w0; s0 < nshort; s0 += 4 * waves) {
        uint64_t i = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t sk = (uint32_t)s0 + (uint32_t)k;
            const int p = 63 - __clzll(__ballot(!lo_half && excl <= sk) >> 32);
            const uint64_t ik = (uint64_t)p * pcap + (sk - (uint32_t)__builtin_amdgcn_readlane((int)excl, 32 + p));
            if (q == k) i = ik;
        }
        const bool mine = s0 + (uint64_t)q < nshort;
        uint64_t src = 0, dst = 0;
        uint32_t len = 0, req = 0;
        if (mine) {
            src = sh[i].src;
            dst = sh[i].dst;
            len = sh[i].len;
            req = sh[i].req;
        }
        copy_span<16>((uint8_t *)dst, (const uint8_t *)src, len, nt, l);
        if (mine && b.t_done && l == 0) {
            uint32_t old = atomicSub(&b.pending[req], 1u);
            if (old == 1) b.t_done[req] = now_ns(b);
        }
    }
}

// Spill pass of one epoch: the groups whose runs did not all fit the queues
// while translation ran during an earlier epoch's copies.  Launched after the
// previous epoch's copy and this epoch's translation, and before the next
// epoch's copy, so that it runs beside the epoch's own copy: every payload
// byte still moves in epoch order.  Each group is translated again (same
// results: page tables change only in A/D bits, which are OR-ed) and its
// wavefront copies every run of it; a run the copy kernel also moves gets the
// same bytes twice, since nothing else in the epoch touches them (batch
// precondition).
__global__ void __launch_bounds__(256) k_spill(DView v, DBatch b, uint64_t r0, uint64_t r1, uint32_t epoch) {
    extern __shared__ uint8_t smem[];
    const int wave = threadIdx.x >> 6;
    CEnt *cache = (CEnt *)smem + wave * kCacheWays;
    uint32_t *owner = (uint32_t *)((CEnt *)smem + (blockDim.x >> 6) * kCacheWays) + wave * kCacheWays;
    const uint32_t n = uniform_u32(*gp<const g_u32>(&b.ctr[epoch].spill_n));
    if (n == 0) return;
    if ((threadIdx.x & 63) < kCacheWays) cache[threadIdx.x & 63].key = ~0ull;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    GroupOut st = {0, 0, 0, 0, 0, 0, 0};
    devirt_request dummy = {};
    for (uint64_t i = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (uint64_t)wave; i < n; i += nwaves) {
        const uint64_t e = uniform_u64(gp<const g_u64>(b.spill)[r0 + i]);
        if (e & kSpillOne) {  // a large request, alone
            process_group<false, false>(v, b, e & ~kSpillOne, 1, dummy, epoch, cache, owner, true, kLargeKeep, r0,
                                        b.ctr, st, nullptr);
        } else {  // a group; its large requests spill on their own
            const uint32_t gn = (uint32_t)((r1 - e) < b.group ? (r1 - e) : b.group);
            process_group<false, false>(v, b, e, gn, dummy, epoch, cache, owner, true, kLargeSkip, r0, b.ctr, st,
                                        nullptr);
        }
    }
    flush_counters(b.counters, st);
}

__global__ void __launch_bounds__(64) k_plain(DView v, DBatch b, devirt_request req, int inline_copy) {
    __shared__ CEnt cache[kCacheWays];
    __shared__ uint32_t owner[kCacheWays];
    if (threadIdx.x < kCacheWays) cache[threadIdx.x].key = ~0ull;
    if (threadIdx.x == 0) {
        for (uint32_t k = 0; k < 2 * kQParts; ++k) b.ctr[0].q[k][0] = 0;
        *b.t0 = wall_clock64();
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    GroupOut st = {0, 0, 0, 0, 0, 0, 0};
    process_group<true, false>(v, b, 0, 1, req, 0, cache, owner, inline_copy != 0, kLargeKeep, 0, b.ctr, st, nullptr);
    flush_counters(b.counters, st);
}

// translate-only: one lane per address
// The translate-only kernel's record staging area: 64 records of 24 bytes per
// wavefront, after the walk cache and its owner slots, 16-byte aligned.
constexpr uint32_t kXlatStage = 64 * 24;
__host__ __device__ constexpr size_t xlat_stage_off(uint32_t block) {
    return ((size_t)(block / 64) * kCacheWays * (sizeof(CEnt) + sizeof(uint32_t)) + 15) & ~(size_t)15;
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) k_xlat(DView v, uint32_t asid,
                                                                                     const uint64_t *gvas, uint64_t n,
                                               uint32_t flags, devirt_xlat *out, DCounters *counters) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    CEnt *cache = (CEnt *)smem + wave * kCacheWays;
    uint32_t *owner = (uint32_t *)((CEnt *)smem + (blockDim.x >> 6) * kCacheWays) + wave * kCacheWays;
    // the wavefront's 64 records are staged here and written out as
    // contiguous 16-byte chunks (a record is 24 bytes with sub-dword fields),
    // with non-temporal stores: nothing on the GPU reads them back soon
    uint32_t *stage = (uint32_t *)(smem + xlat_stage_off(blockDim.x)) + wave * (kXlatStage / 4);
    if (lane < kCacheWays) cache[lane].key = ~0ull;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const bool valid_asid = asid < v.nproc;
    DProc p = {0, 0, 4};
    DVm vmv = {};
    vmv.lds_base = kLdsNone;
    vmv.lds_idx = kLdsNone;
    if (valid_asid) p = gp<const DV_GLOBAL DProc>(v.procs)[asid];
    const bool lds = valid_asid && lds_slots_load_one(v, p.vm);  // one process: its VM's slots only
    if (valid_asid) vmv = load_vm(v, p.vm, lds);
    const uint64_t lim = user_limit(p.levels);
    const bool write = (flags & DEVIRT_XLAT_WRITE) != 0;
    const bool set_ad = (flags & DEVIRT_XLAT_SET_AD) != 0;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    unsigned long long hits = 0, misses = 0, atom = 0;
    // the next round's addresses are loaded at the top of this round
    const uint64_t first = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + wave) * 64;
    uint64_t gva_next = first + lane < n ? gp<const g_u64>(gvas)[first + lane] : 0;
    for (uint64_t b0 = first; b0 < n; b0 += waves * 64) {
        const uint64_t i = b0 + lane;
        const bool in = i < n;
        const uint64_t gva = gva_next;
        gva_next = i + waves * 64 < n ? gp<const g_u64>(gvas)[i + waves * 64] : 0;
        devirt_xlat x;
        x.gpa = 0;
        x.hpa = 0;
        x.code = 0;
        x.level = 0;
        x.page_shift = 0;
        x.vm = valid_asid ? (uint16_t)p.vm : (uint16_t)0xFFFF;
        bool go = in && valid_asid;
        if (in && !valid_asid) x.code = DEVIRT_INVALID;
        if (go && gva >= lim) {
            x.code = DEVIRT_NONCANONICAL;
            go = false;
        }
        CEnt ce;
        ce.info = 0;
        ce.path[0] = ce.path[1] = ce.path[2] = 0;
        ce.base = 0;
        uint32_t cslot;
        bool chit;
        cache_resolve(cache, owner, go, ((uint64_t)asid << 27) | (gva >> 30), vmv, p.cr3, p.levels, gva, ce, cslot,
                      chit);
        if (go) {
            if (chit)
                hits++;
            else
                misses++;
            uint32_t code = ci_code(ce.info), level = ci_level(ce.info);
            uint32_t u = ci_u(ce.info), w = ci_w(ce.info), leaf_level = 0, shift = 0;
            uint64_t frame = 0, pde_off = 0, pte_off = 0, e2 = 0, e1 = 0;
            if (code == 0) {
                if (ci_leaf(ce.info)) {
                    frame = ce.base;
                    shift = 30;
                    leaf_level = 3;
                } else {
                    uint64_t th;
                    const uint32_t xc = gpa_xlat(vmv, ce.base, kNeedTable, th);
                    if (xc) {
                        code = xc;
                        level = 2;
                    } else {
                        pde_off = th + 8 * ((gva >> 21) & 511);
                        e2 = load_entry(vmv.arena, pde_off);
                        if (!(e2 & kP)) {
                            code = DEVIRT_NOT_PRESENT;
                            level = 2;
                        } else if (p.levels == 3 && (e2 & kPaeRsvd)) {
                            code = DEVIRT_RESERVED;
                            level = 2;
                        } else {
                            u &= (uint32_t)(e2 >> 2) & 1u;
                            w &= (uint32_t)(e2 >> 1) & 1u;
                            if (e2 & kPS) {
                                if (e2 & 0x1FE000ull) {
                                    code = DEVIRT_RESERVED;
                                    level = 2;
                                } else {
                                    frame = e2 & kAddrMask & ~((1ull << 21) - 1);
                                    shift = 21;
                                    leaf_level = 2;
                                }
                            } else {
                                uint64_t pt;
                                const uint32_t xc1 = gpa_xlat(vmv, e2 & kAddrMask, kNeedTable, pt);
                                if (xc1) {
                                    code = xc1;
                                    level = 1;
                                } else {
                                    pte_off = pt + 8 * ((gva >> 12) & 511);
                                    e1 = load_entry(vmv.arena, pte_off);
                                    if (!(e1 & kP)) {
                                        code = DEVIRT_NOT_PRESENT;
                                        level = 1;
                                    } else if (p.levels == 3 && (e1 & kPaeRsvd)) {
                                        code = DEVIRT_RESERVED;
                                        level = 1;
                                    } else {
                                        u &= (uint32_t)(e1 >> 2) & 1u;
                                        w &= (uint32_t)(e1 >> 1) & 1u;
                                        frame = e1 & kAddrMask;
                                        shift = 12;
                                        leaf_level = 1;
                                    }
                                }
                            }
                        }
                    }
                }
            }
            uint64_t gpa = 0, hpa = 0;
            if (code == 0) {
                gpa = frame | (gva & ((1ull << shift) - 1));
                x.gpa = gpa;
                x.page_shift = (uint8_t)shift;
                if (!u) {
                    code = DEVIRT_PROT_USER;
                    level = leaf_level;
                } else if (write && !w) {
                    code = DEVIRT_PROT_WRITE;
                    level = leaf_level;
                } else {
                    const uint32_t xc = gpa_xlat(vmv, gpa, write ? kNeedW : kNeedR, hpa);
                    if (xc) {
                        code = xc;
                        level = 0;
                        hpa = 0;
                    }
                }
            }
            x.code = code;
            x.level = (uint8_t)level;
            if (code == 0) {
                x.hpa = hpa;
                if (set_ad) {
                    const uint32_t np = ci_np(ce.info), ab = ci_abits(ce.info);
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        if ((uint32_t)q >= np) continue;
                        uint32_t want = (uint32_t)kA;
                        bool need = !((ab >> q) & 1u);
                        if (leaf_level == 3 && (uint32_t)q + 1 == np && write) {
                            want |= (uint32_t)kD;
                            need = need || !(ce.info & kCiDbit);
                        }
                        if (need) {
                            or_entry(vmv.arena, ce.path[q], want);
                            atom++;
                        }
                    }
                    if (leaf_level <= 2) {
                        uint32_t want = (uint32_t)kA | ((leaf_level == 2 && write) ? (uint32_t)kD : 0u);
                        if (((uint32_t)e2 & want) != want) {
                            or_entry(vmv.arena, pde_off, want);
                            atom++;
                        }
                    }
                    if (leaf_level == 1) {
                        uint32_t want = (uint32_t)kA | (write ? (uint32_t)kD : 0u);
                        if (((uint32_t)e1 & want) != want) {
                            or_entry(vmv.arena, pte_off, want);
                            atom++;
                        }
                    }
                }
            }
        }
        // every lane stages its record (an idle lane's is never written out)
        {
            uint32_t *r = stage + 6 * lane;
            *(uint64_t *)r = x.gpa;
            *(uint64_t *)(r + 2) = x.hpa;
            r[4] = x.code;
            r[5] = (uint32_t)x.level | ((uint32_t)x.page_shift << 8) | ((uint32_t)x.vm << 16);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        {
            const uint32_t valid = 24u * (uint32_t)(n - b0 < 64 ? n - b0 : 64);  // bytes of this round
            uint8_t *dst = (uint8_t *)out + 24 * b0;
#pragma unroll
            for (uint32_t k = 0; k < 2; ++k) {
                const uint32_t c = (uint32_t)lane + 64u * k;  // 16-byte chunk of the round
                if (16u * c + 16u <= valid)
                    __builtin_nontemporal_store(*(const u32x4 *)(stage + 4 * c), gp<g_u32x4_w4>(dst + 16 * c));
                else if (16u * c < valid)  // the last 8 bytes of an odd count
                    __builtin_nontemporal_store(*(const uint64_t *)(stage + 4 * c), gp<g_u64>(dst + 16 * c));
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    if (counters) {
        GroupOut st = {0, hits, misses, 0, 0, atom, 0};
        flush_counters(counters, st);
    }
}

// ------------------------------------------------------------ fault list
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t *lds, uint32_t &total) {
    const int lane = lane_id(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = shfl32(incl, lane >= d ? lane - d : lane);
        if (lane >= d) incl += t;
    }
    if (lane == 63) lds[wave] = incl;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int w = 0; w < nw; ++w) {
        uint32_t s = lds[w];
        if (w < wave) before += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return before + incl - x;
}

__global__ void __launch_bounds__(256) k_fault_count(const devirt_result *res, uint64_t n, uint32_t *tile_cnt) {
    __shared__ uint32_t lds[16];
    const uint64_t t = blockIdx.x;
    uint32_t c = 0;
    for (int q = 0; q < 4; ++q) {
        uint64_t i = t * kFaultTile + (uint64_t)threadIdx.x * 4 + q;
        if (i < n && res[i].code != 0) c++;
    }
    uint32_t tot;
    block_exclusive_scan(c, lds, tot);
    if (threadIdx.x == 0) tile_cnt[t] = tot;
}

__global__ void __launch_bounds__(1024) k_fault_scan(uint32_t *tile_cnt, uint64_t ntiles, uint64_t *n_faults) {
    __shared__ uint32_t lds[16];
    uint64_t carry = 0;
    for (uint64_t b0 = 0; b0 < ntiles; b0 += blockDim.x) {
        const uint64_t i = b0 + threadIdx.x;
        const uint32_t x = i < ntiles ? tile_cnt[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(x, lds, tot);
        if (i < ntiles) tile_cnt[i] = (uint32_t)(carry + ex);
        carry += tot;
    }
    if (threadIdx.x == 0 && n_faults) *n_faults = carry;
}

__global__ void __launch_bounds__(256) k_fault_scatter(const devirt_result *res, uint64_t n, const uint32_t *tile_off,
                                                       devirt_fault *faults) {
    __shared__ uint32_t lds[16];
    const uint64_t t = blockIdx.x;
    uint32_t flags = 0, c = 0;
    for (int q = 0; q < 4; ++q) {
        uint64_t i = t * kFaultTile + (uint64_t)threadIdx.x * 4 + q;
        if (i < n && res[i].code != 0) {
            flags |= 1u << q;
            c++;
        }
    }
    uint32_t tot;
    uint32_t pos = tile_off[t] + block_exclusive_scan(c, lds, tot);
    for (int q = 0; q < 4; ++q) {
        if (flags & (1u << q)) {
            uint64_t i = t * kFaultTile + (uint64_t)threadIdx.x * 4 + q;
            devirt_result r = res[i];
            devirt_fault f;
            f.req_index = i;
            f.fault_gva = r.fault_gva;
            f.code = r.code;
            f.level = r.level;
            f.pad = 0;
            faults[pos++] = f;
        }
    }
}

// ---------------------------------------------------------------- launchers
static size_t wave_lds(int block) {
    return (size_t)(block / 64) * kCacheWays * (sizeof(CEnt) + sizeof(uint32_t));
}

hipError_t launch_reset(hipStream_t s, DBatch b, uint32_t n_epochs) {
    uint32_t blocks = (n_epochs + 255) / 256;
    if (blocks == 0) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_reset, dim3(blocks), dim3(256), 0, s, b, n_epochs);
    return hipGetLastError();
}

hipError_t launch_translate_groups(hipStream_t s, int grid, int block, DView v, DBatch b, uint64_t r0, uint64_t r1,
                                   uint32_t epoch, int direct) {
    hipLaunchKernelGGL(k_translate_groups, dim3(grid), dim3(block), wave_lds(block), s, v, b, r0, r1, epoch, direct);
    return hipGetLastError();
}

hipError_t launch_translate_large(hipStream_t s, int grid, int block, DView v, DBatch b, uint64_t r0,
                                  uint32_t epoch) {
    hipLaunchKernelGGL(k_translate_large, dim3(grid), dim3(block), wave_lds(block), s, v, b, r0, epoch);
    return hipGetLastError();
}

hipError_t launch_copy(hipStream_t s, int grid, int block, DBatch b, uint32_t epoch) {
    hipLaunchKernelGGL(k_copy, dim3(grid), dim3(block), 0, s, b, epoch);
    return hipGetLastError();
}

hipError_t launch_spill(hipStream_t s, int grid, int block, DView v, DBatch b, uint64_t r0, uint64_t r1,
                        uint32_t epoch) {
    hipLaunchKernelGGL(k_spill, dim3(grid), dim3(block), wave_lds(block), s, v, b, r0, r1, epoch);
    return hipGetLastError();
}

hipError_t launch_plain(hipStream_t s, DView v, DBatch b, devirt_request req, int inline_copy) {
    hipLaunchKernelGGL(k_plain, dim3(1), dim3(64), 0, s, v, b, req, inline_copy);
    return hipGetLastError();
}

hipError_t launch_xlat(hipStream_t s, int grid, int block, DView v, uint32_t asid, const uint64_t *gva, uint64_t n,
                       uint32_t flags, devirt_xlat *out, DCounters *counters) {
    hipLaunchKernelGGL(k_xlat, dim3(grid), dim3(block), xlat_stage_off(block) + (size_t)(block / 64) * kXlatStage, s, v,
                       asid, gva, n, flags, out, counters);
    return hipGetLastError();
}

hipError_t launch_fault_count(hipStream_t s, const devirt_result *res, uint64_t n, uint32_t *tile_cnt) {
    uint64_t tiles = (n + kFaultTile - 1) / kFaultTile;
    if (tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fault_count, dim3((unsigned)tiles), dim3(256), 0, s, res, n, tile_cnt);
    return hipGetLastError();
}

hipError_t launch_fault_scan(hipStream_t s, uint32_t *tile_cnt, uint64_t ntiles, uint64_t *n_faults) {
    hipLaunchKernelGGL(k_fault_scan, dim3(1), dim3(1024), 0, s, tile_cnt, ntiles, n_faults);
    return hipGetLastError();
}

hipError_t launch_fault_scatter(hipStream_t s, const devirt_result *res, uint64_t n, const uint32_t *tile_off,
                                devirt_fault *faults) {
    uint64_t tiles = (n + kFaultTile - 1) / kFaultTile;
    if (tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fault_scatter, dim3((unsigned)tiles), dim3(256), 0, s, res, n, tile_off, faults);
    return hipGetLastError();
}


// ------------------------------------------------------------- map pages
// Mapping pages by writing the guest's own tables (section 4.2, the second
// kind of routine).  Keys name tables: (8 - level) in bits 63:56, the table's
// index (gva >> (12 + 9 level)) below, so ascending keys run from the top
// level down and by index within a level.
__device__ __forceinline__ uint64_t map_key(uint32_t level, uint64_t gva) {
    return ((uint64_t)(8 - level) << 56) | (gva >> (12 + 9 * level));
}

// Index of gva's entry in its table at `level` (a PAE root table has 4).
__device__ __forceinline__ uint64_t entry_index(uint32_t levels, uint32_t level, uint64_t gva) {
    return (levels == 3 && level == 3) ? ((gva >> 30) & 3) : ((gva >> (12 + 9 * (level - 1))) & 511);
}

__device__ __forceinline__ uint64_t root_table(const DProc &p) {
    return p.levels == 3 ? (p.cr3 & 0xFFFFFFE0ull) : (p.cr3 & kAddrMask);
}

__device__ __forceinline__ void store_entry(uint8_t *arena, uint64_t off, uint64_t v) { *gp<g_u64>(arena + off) = v; }

// Walk for a map on the tables as they are (no A/D).  On success `missing` is
// the highest level whose entry is not present (its child tables are lacking),
// 0 when the whole path exists.
__device__ uint32_t map_walk(const DVm &v, const DProc &p, uint64_t gva, uint32_t &level, uint32_t &missing) {
    const bool pae = p.levels == 3;
    uint64_t table = root_table(p);
    missing = 0;
    for (int lvl = (int)p.levels; lvl >= 2; --lvl) {
        uint64_t th;
        const uint32_t xc = gpa_xlat(v, table, kNeedTable, th);
        if (xc) {
            level = (uint32_t)lvl;
            return xc;
        }
        const uint64_t e = load_entry(v.arena, th + 8 * entry_index(p.levels, (uint32_t)lvl, gva));
        if (!(e & kP)) {
            missing = (uint32_t)lvl;
            return DEVIRT_OK;
        }
        const bool root = pae && lvl == 3;
        const bool rsvd = pae && (e & (root ? kPaeRootRsvd : kPaeRsvd)) != 0;
        if (rsvd || (!root && (e & kPS))) {  // reserved bits, or a large leaf on the path
            level = (uint32_t)lvl;
            return DEVIRT_RESERVED;
        }
        table = e & kAddrMask;
    }
    uint64_t th;
    const uint32_t xc = gpa_xlat(v, table, kNeedTable, th);  // the page table itself
    if (xc) {
        level = 1;
        return xc;
    }
    return DEVIRT_OK;
}

// Arena offset of the existing table at `level` on gva's path (the path to it
// is known to be present); level == top gives the root table.  False if a
// table on the way has no memslot (then nothing may be written).
__device__ bool existing_table(const DVm &v, const DProc &p, uint64_t gva, uint32_t level, uint64_t &th) {
    uint64_t table = root_table(p);
    for (int lvl = (int)p.levels; lvl > (int)level; --lvl) {
        if (gpa_xlat(v, table, kNeedTable, th)) return false;
        table = load_entry(v.arena, th + 8 * entry_index(p.levels, (uint32_t)lvl, gva)) & kAddrMask;
    }
    return gpa_xlat(v, table, kNeedTable, th) == DEVIRT_OK;
}

// ---- the EPT half of mapping a page (section 4.2: the backend creates the
// mapping in the guest tables and also in the EPT), devirt_ept_map_pages.
// The maps name guest-physical pages and the arena pages behind them; new EPT
// tables are linked with R, W and X, leaves carry the map's R/W/X bits and
// memory type WB.
constexpr uint64_t kEptRwx = 7ull, kEptWb = 6ull << 3;

__device__ __forceinline__ uint64_t ept_slot(uint64_t table, uint32_t level, uint64_t gpa) {
    return table + 8 * ((gpa >> (12 + 9 * (level - 1))) & 511);
}

// Walk of the EPT as it is, for a map of gpa.  On success `missing` is the
// highest level whose entry is not present (its child tables are lacking), 0
// when the EPT page table exists.  A present large leaf on the path fails the
// map (RESERVED: nothing is split), a misconfigured table entry or a table
// outside the arena fails it with EPT_MISCONFIG; `level` names the entry.
__device__ uint32_t ept_map_walk(const DVm &v, uint64_t gpa, uint32_t &level, uint32_t &missing) {
    uint64_t table = v.ept_root;
    missing = 0;
    for (uint32_t lvl = 4; lvl >= 2; --lvl) {
        const uint64_t e = load_entry(v.arena, ept_slot(table, lvl, gpa));
        if (!(e & 7)) {
            missing = lvl;
            level = 0;
            return DEVIRT_OK;
        }
        level = lvl;
        if ((e & 3) == 2) return DEVIRT_EPT_MISCONFIG;  // write without read
        if (lvl <= 3 && (e & 0x80)) return DEVIRT_RESERVED;
        if (e & 0xF8) return DEVIRT_EPT_MISCONFIG;  // bits 7:3 of a table entry
        table = e & kAddrMask;
        if (table >= v.arena_bytes || v.arena_bytes - table < 4096) return DEVIRT_EPT_MISCONFIG;
    }
    level = 0;
    return DEVIRT_OK;
}

// Arena offset of the existing EPT table at `level` on gpa's path (known present).
__device__ uint64_t existing_ept_table(const DVm &v, uint64_t gpa, uint32_t level) {
    uint64_t table = v.ept_root;
    for (uint32_t lvl = 4; lvl > level; --lvl) table = load_entry(v.arena, ept_slot(table, lvl, gpa)) & kAddrMask;
    return table;
}

// Position of key in the sorted keys[0, n), or -1.
__device__ __forceinline__ int64_t find_key(const uint64_t *keys, uint64_t n, uint64_t key) {
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (keys[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < n && keys[lo] == key) ? (int64_t)lo : -1;
}

// Fibonacci hashing (Knuth): the top log2 bits of key * 2^64/phi.
__device__ __forceinline__ uint64_t hash_slot(uint64_t key, uint32_t log2) {
    return (key * 0x9E3779B97F4A7C15ull) >> (64 - log2);
}

// Adds a table key to the set, probing from slot h (the key's probe number
// `probe` there); its first inserter also appends it to the list tkeys[0, m).
// sc[0] counts distinct keys.  A long probe chain gives up, with sc[3] set,
// once more than m distinct keys exist: the set holds at least twice m + 1
// slots, so chains grow long only then, and the count (an address every new
// key increments, so reads of it serialize) is read only on such chains.
// Every probe loop is bounded by the set's size.
constexpr uint64_t kLongChain = 8;
__device__ void tset_insert_from(const MapArgs &a, uint64_t key, uint64_t h, uint64_t probe) {
    const uint64_t mask = (1ull << a.tset_log2) - 1;
    for (; probe <= mask; ++probe) {
        const uint64_t cur = atomicCAS((unsigned long long *)&a.tset[h], ~0ull, (unsigned long long)key);
        if (cur == ~0ull) {
            const uint64_t idx = atomicAdd((unsigned long long *)&a.sc[0], 1ull);
            if (idx < a.m) a.tkeys[idx] = key;
            return;
        }
        if (cur == key) return;
        if (probe >= kLongChain && __hip_atomic_load(&a.sc[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > a.m)
            break;
        h = (h + 1) & mask;
    }
    __hip_atomic_store(&a.sc[3], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A lane's (up to four) table keys: the first probes are issued together, so
// the lane waits for one atomic round trip, not one per key; a key whose first
// slot holds another key continues in tset_insert_from.
__device__ void tset_insert4(const MapArgs &a, const uint64_t (&key)[4], const bool (&want)[4]) {
    const uint64_t mask = (1ull << a.tset_log2) - 1;
    uint64_t h[4], cur[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        h[j] = hash_slot(key[j], a.tset_log2);
        cur[j] = want[j] ? (uint64_t)atomicCAS((unsigned long long *)&a.tset[h[j]], ~0ull,
                                               (unsigned long long)key[j])
                         : key[j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (!want[j] || cur[j] == key[j]) continue;
        if (cur[j] == ~0ull) {
            const uint64_t idx = atomicAdd((unsigned long long *)&a.sc[0], 1ull);
            if (idx < a.m) a.tkeys[idx] = key[j];
        } else {
            tset_insert_from(a, key[j], (h[j] + 1) & mask, 1);
        }
    }
}

// Records map i for its page: a slot holds (page << kMapIdxBits | index), and
// a later map of the same page raises it with atomicMax, so the slot ends up
// naming the page's last map.  A page seen once costs one atomic.  The set
// has at least twice as many slots as maps, so a free slot is always found.
__device__ void page_note(const MapArgs &a, uint64_t page, uint64_t i) {
    const uint64_t mask = (1ull << a.pset_log2) - 1;
    const uint64_t v = (page << kMapIdxBits) | i;
    uint64_t h = hash_slot(page, a.pset_log2);
    for (uint64_t probe = 0; probe <= mask; ++probe) {
        const uint64_t cur = atomicCAS((unsigned long long *)&a.pset[h], ~0ull, (unsigned long long)v);
        if (cur == ~0ull) return;
        if ((cur >> kMapIdxBits) == page) {
            atomicMax((unsigned long long *)&a.pset[h], (unsigned long long)v);
            return;
        }
        h = (h + 1) & mask;
    }
}

// Fill `ones` with ~0 (empty set slots, list padding) and `zeros` with 0.
__global__ void __launch_bounds__(256) k_map_clear(uint64_t *ones, uint64_t n_ones, uint64_t *zeros, uint64_t n_zeros) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_ones + n_zeros; t += stride) {
        if (t < n_ones)
            ones[t] = ~0ull;
        else
            zeros[t - n_ones] = 0;
    }
}

// One lane per map: its result; the tables its path lacks go into the set
// (a key the previous lane of the wavefront holds in the same position is
// left to that lane); a successful map is noted for its page.
__global__ void __launch_bounds__(256) k_map_walk(MapArgs a) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < a.n;
    uint64_t k[4] = {~0ull, ~0ull, ~0ull, ~0ull};
    uint64_t gva = 0;
    bool ok = false;
    if (live) {
        const devirt_map m = a.maps[i];
        gva = m.gva;
        devirt_result r;
        r.bytes_done = 0;
        r.fault_gva = m.gva;
        r.code = DEVIRT_OK;
        r.level = 0;
        r.pad = 0;
        if (a.ept_map) {  // gva: the guest-physical page; gpa: the arena page behind it
            const DVm vm = a.v.vms[a.vm];
            const uint32_t perms = m.flags & 7u;
            if ((m.gva & 0xFFFull) || (m.gva >> 48) || (m.gpa & 0xFFFull) || m.gpa >= vm.arena_bytes ||
                vm.arena_bytes - m.gpa < 4096 || (m.flags & ~7u) || perms == 0 || (perms & 3u) == 2u) {
                r.code = DEVIRT_NONCANONICAL;
            } else {
                uint32_t level = 0, missing = 0;
                r.code = ept_map_walk(vm, m.gva, level, missing);
                r.level = (uint16_t)level;
                if (r.code == DEVIRT_OK) {
                    r.bytes_done = 4096;
                    r.fault_gva = 0;
                    ok = true;
                    int j = 0;
                    for (uint32_t l = missing ? missing - 1 : 0; l >= 1 && j < 4; --l) k[j++] = map_key(l, m.gva);
                }
            }
        } else if (a.asid >= a.v.nproc) {
            r.code = DEVIRT_INVALID;
        } else {
            const DProc p = a.v.procs[a.asid];
            const DVm vm = a.v.vms[p.vm];
            if ((m.gva & 0xFFFull) || m.gva >= user_limit(p.levels) || (m.gpa & 0xFFFull) || m.gpa >= (1ull << 52)) {
                r.code = DEVIRT_NONCANONICAL;
            } else {
                uint32_t level = 0, missing = 0;
                r.code = map_walk(vm, p, m.gva, level, missing);
                r.level = (uint16_t)level;
                if (r.code == DEVIRT_OK) {
                    r.bytes_done = 4096;
                    r.fault_gva = 0;
                    ok = true;
                    int j = 0;
                    for (uint32_t l = missing ? missing - 1 : 0; l >= 1 && j < 4; --l) k[j++] = map_key(l, m.gva);
                }
            }
        }
        a.res[i] = r;
    }
    const int lane = lane_id();
    bool want[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint64_t prev = shfl64(k[j], lane > 0 ? lane - 1 : 0);
        want[j] = k[j] != ~0ull && (lane == 0 || prev != k[j]);
    }
    tset_insert4(a, k, want);
    if (ok) page_note(a, gva >> 12, i);
}

// A VM with an EPT: the pool frames the batch takes (the first sc[0]) are
// translated through the EPT, readable and writable like every table frame;
// one that is not makes the batch fail as a short pool does (sc[3]).
__global__ void __launch_bounds__(256) k_map_pool(const MapArgs a) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nt = a.sc[0];
    if (a.sc[3] || nt > a.n_pool || k >= nt || a.asid >= a.v.nproc) return;
    const DVm vm = a.v.vms[a.v.procs[a.asid].vm];
    uint64_t h = 0;
    if (gpa_xlat(vm, a.pool_gpa[k], kNeedTable, h) == DEVIRT_OK)
        a.pool_hpa[k] = h;
    else
        __hip_atomic_store(&a.sc[3], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The VM whose tables a map call writes (false: an unknown asid).
__device__ __forceinline__ bool map_vm(const MapArgs &a, DVm &vm) {
    if (a.ept_map) {
        vm = a.v.vms[a.vm];
        return true;
    }
    if (a.asid >= a.v.nproc) return false;
    vm = a.v.vms[a.v.procs[a.asid].vm];
    return true;
}

// Tables to create: 0 when the pool is too small (then nothing is written).
__device__ __forceinline__ uint64_t new_tables(const MapArgs &a) {
    const uint64_t u = a.sc[0];
    return (a.sc[3] != 0 || u > a.n_pool) ? 0 : u;
}
__device__ __forceinline__ bool pool_short(const MapArgs &a) { return a.sc[3] != 0 || a.sc[0] > a.n_pool; }

// The distinct keys are sorted by rank (the number of smaller keys; there are
// no ties), in LDS tiles: for lists of up to kMapRankMax keys.  The same
// launch zeroes the new tables, 16 bytes per lane.
__global__ void __launch_bounds__(256) k_map_rank_zero(const MapArgs a) {
    __shared__ uint64_t tile[256];
    const uint64_t nt = new_tables(a);
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    DVm zvm;
    if (nt && map_vm(a, zvm)) {
        uint8_t *arena = zvm.arena;
        const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
        for (uint64_t z = t; z < nt * 256; z += stride)
            *gp<g_u32x4>(arena + a.pool_hpa[z >> 8] + 16 * (z & 255)) = (u32x4){0u, 0u, 0u, 0u};
    }
    if (!a.rank || (uint64_t)blockIdx.x * blockDim.x >= nt) return;  // uniform per block
    const uint64_t key = t < nt ? a.tkeys[t] : ~0ull;
    uint64_t rank = 0;
    for (uint64_t base = 0; base < nt; base += 256) {
        __syncthreads();
        tile[threadIdx.x] = base + threadIdx.x < nt ? a.tkeys[base + threadIdx.x] : ~0ull;
        __syncthreads();
        const uint32_t cnt = (uint32_t)std::min<uint64_t>(256, nt - base);
        for (uint32_t q = 0; q < cnt; ++q) rank += tile[q] < key;
    }
    if (t < nt) a.tkeys_sorted[rank] = key;
}

// Longer key lists (more than kMapRankMax keys can exist) are sorted in two
// steps.  First tiles of kSortTile keys, each by rank in LDS; then rounds of
// pairwise merges of sorted runs, in which a key's place in the merged run is
// its place in its own run plus the number of smaller keys in the other run,
// found by a binary search of that run.  Only the list's first
// min(sc[0], m) entries are keys, all distinct, so there are no ties; the
// rest is never read.  The steps alternate between tkeys and tkeys_sorted.
constexpr uint32_t kSortTile = 1024;

__device__ __forceinline__ uint64_t sort_count(const MapArgs &a) { return a.sc[0] < a.m ? a.sc[0] : a.m; }

__global__ void __launch_bounds__(256) k_map_tile_sort(const MapArgs a, const uint64_t *src, uint64_t *dst) {
    static_assert(kSortTile % 256 == 0, "a tile is a whole number of keys per lane");
    __shared__ uint64_t tile[kSortTile];
    const uint64_t cnt = sort_count(a);
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    if (base >= cnt) return;  // uniform per block
    const uint32_t len = (uint32_t)std::min<uint64_t>(kSortTile, cnt - base);
    for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) tile[i] = src[base + i];
    __syncthreads();  // src may be dst: every read of the tile is done
    // each lane ranks its kSortTile / 256 keys in one sweep of the tile; a
    // lane past the tile's end ranks the largest key, and its rank is not used
    constexpr uint32_t K = kSortTile / 256;
    uint64_t key[K];
    uint32_t rank[K];
#pragma unroll
    for (uint32_t j = 0; j < K; ++j) {
        key[j] = ~0ull;
        rank[j] = 0;
        if (threadIdx.x + 256 * j < len) key[j] = tile[threadIdx.x + 256 * j];
    }
    for (uint32_t q = 0; q < len; ++q) {
        const uint64_t t = tile[q];
#pragma unroll
        for (uint32_t j = 0; j < K; ++j) rank[j] += t < key[j];
    }
#pragma unroll
    for (uint32_t j = 0; j < K; ++j)
        if (threadIdx.x + 256 * j < len) dst[base + rank[j]] = key[j];
}

// One merge round: runs of w keys (a power of two, at least kSortTile) are
// merged in pairs.
__global__ void __launch_bounds__(256) k_map_merge(const MapArgs a, const uint64_t *src, uint64_t *dst, uint64_t w) {
    const uint64_t cnt = sort_count(a);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride) {
        const uint64_t key = src[i];
        const uint64_t pair = i & ~(2 * w - 1);
        const bool second = (i & w) != 0;
        const uint64_t own = second ? pair + w : pair;
        const uint64_t other = second ? pair : pair + w;
        const uint64_t olen = other >= cnt ? 0 : std::min<uint64_t>(w, cnt - other);
        uint64_t lo = 0, hi = olen;  // smaller keys in the other run: [0, lo)
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (src[other + mid] < key)
                lo = mid + 1;
            else
                hi = mid;
        }
        dst[pair + (i - own) + lo] = key;
    }
}

// Zero the new tables (after a long list's sort).
__global__ void __launch_bounds__(256) k_map_zero(const MapArgs a) {
    const uint64_t nt = new_tables(a);
    DVm zvm;
    if (!nt || !map_vm(a, zvm)) return;
    uint8_t *arena = zvm.arena;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt * 256; t += stride)
        *gp<g_u32x4>(arena + a.pool_hpa[t >> 8] + 16 * (t & 255)) = (u32x4){0u, 0u, 0u, 0u};
}

// Lane t links new table t (sorted position t takes pool frame t) from its
// parent entry, in a new table or an existing one, and handles map t: NO_POOL
// when the pool is short, else the leaf if it is the last map of its page.
// Links and leaves touch disjoint entries: a leaf whose page table exists has
// a fully present path, and links write only not-present entries (in existing
// tables) or entries of new tables.
__global__ void __launch_bounds__(256) k_map_write(const MapArgs a) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool short_pool = pool_short(a);
    const uint64_t nt = short_pool ? 0 : a.sc[0];
    if (t == 0) *a.n_used = nt;
    const uint64_t *uniq = a.tkeys_sorted;
    if (a.ept_map) {
        const DVm vm = a.v.vms[a.vm];
        if (t < nt) {  // link new EPT table t from its parent (new, or existing above it)
            const uint64_t key = uniq[t];
            const uint32_t l = 8u - (uint32_t)(key >> 56);
            const uint64_t gpa = (key & ((1ull << 56) - 1)) << (12 + 9 * l);
            const int64_t j = l + 1 < 4 ? find_key(uniq, nt, map_key(l + 1, gpa)) : -1;
            const uint64_t parent = j >= 0 ? a.pool_hpa[j] : existing_ept_table(vm, gpa, l + 1);
            store_entry(vm.arena, ept_slot(parent, l + 1, gpa), a.pool_hpa[t] | kEptRwx);
        }
        if (t >= a.n || a.res[t].code != DEVIRT_OK) return;
        const devirt_map m = a.maps[t];
        if (short_pool) {
            a.res[t].code = DEVIRT_NO_POOL;
            a.res[t].bytes_done = 0;
            a.res[t].fault_gva = m.gva;
            return;
        }
        const uint64_t page = m.gva >> 12;
        const uint64_t mask = (1ull << a.pset_log2) - 1;
        uint64_t h = hash_slot(page, a.pset_log2);
        for (uint64_t probe = 0; probe <= mask && (a.pset[h] >> kMapIdxBits) != page; ++probe) h = (h + 1) & mask;
        if (a.pset[h] != ((page << kMapIdxBits) | t)) return;  // not the page's last map
        const int64_t j = find_key(uniq, nt, map_key(1, m.gva));
        const uint64_t pt = j >= 0 ? a.pool_hpa[j] : existing_ept_table(vm, m.gva, 1);
        store_entry(vm.arena, ept_slot(pt, 1, m.gva), m.gpa | (m.flags & 7u) | kEptWb);
        return;
    }
    if (a.asid >= a.v.nproc) return;
    const DProc p = a.v.procs[a.asid];
    const DVm vm = a.v.vms[p.vm];
    if (t < nt) {
        const uint64_t key = uniq[t];
        const uint32_t l = 8u - (uint32_t)(key >> 56);
        const uint64_t id = key & ((1ull << 56) - 1);
        const uint64_t va = id << (12 + 9 * l);
        int64_t j = -1;
        if (l + 1 < p.levels) j = find_key(uniq, nt, map_key(l + 1, va));
        uint64_t phpa = 0;
        bool have = true;
        if (j >= 0)
            phpa = a.pool_hpa[j];
        else
            have = existing_table(vm, p, va, l + 1, phpa);
        if (have) {
            const bool root_pae = p.levels == 3 && l + 1 == 3;
            const uint64_t idx = root_pae ? ((va >> 30) & 3) : (id & 511);
            store_entry(vm.arena, phpa + 8 * idx, a.pool_gpa[t] | (root_pae ? kP : (kP | kRW | kUS)));
        }
    }
    if (t >= a.n || a.res[t].code != DEVIRT_OK) return;
    const devirt_map m = a.maps[t];
    if (short_pool) {
        a.res[t].code = DEVIRT_NO_POOL;
        a.res[t].bytes_done = 0;
        a.res[t].fault_gva = m.gva;
        return;
    }
    const uint64_t page = m.gva >> 12;
    const uint64_t mask = (1ull << a.pset_log2) - 1;
    uint64_t h = hash_slot(page, a.pset_log2);
    for (uint64_t probe = 0; probe <= mask && (a.pset[h] >> kMapIdxBits) != page; ++probe) h = (h + 1) & mask;
    if (a.pset[h] != ((page << kMapIdxBits) | t)) return;  // not the page's last map
    const int64_t j = find_key(uniq, nt, map_key(1, m.gva));
    uint64_t pt = 0;
    if (j >= 0)
        pt = a.pool_hpa[j];
    else if (!existing_table(vm, p, m.gva, 1, pt))
        return;
    store_entry(vm.arena, pt + 8 * ((m.gva >> 12) & 511), m.gpa | kP | kUS | ((m.flags & DEVIRT_MAP_WRITE) ? kRW : 0ull));
}

static unsigned blocks_for(uint64_t n) { return (unsigned)((n + 255) / 256 ? (n + 255) / 256 : 1); }

hipError_t launch_map(hipStream_t s, const MapArgs &a) {
    hipError_t e;
    const uint64_t nset = (1ull << a.tset_log2), npset = (1ull << a.pset_log2);
    // tset, tkeys and pset are contiguous, then sc
    const uint64_t ones = nset + a.m + npset, zeros = 4;
    hipLaunchKernelGGL(k_map_clear, dim3(blocks_for(std::min<uint64_t>(ones + zeros, 1ull << 22))), dim3(256), 0, s,
                       a.tset, ones, a.sc, zeros);
    hipLaunchKernelGGL(k_map_walk, dim3(blocks_for(a.n)), dim3(256), 0, s, a);
    if (a.ept_pool) hipLaunchKernelGGL(k_map_pool, dim3(blocks_for(a.m)), dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (a.rank) {
        // enough lanes to zero every possible new table in one sweep (at most 2^22)
        hipLaunchKernelGGL(k_map_rank_zero, dim3(blocks_for(std::max(a.m, std::min<uint64_t>(a.m * 256, 1ull << 22)))),
                           dim3(256), 0, s, a);
    } else {
        // merge rounds for m keys; the tile sort's output buffer is chosen so
        // that the last round writes tkeys_sorted
        uint32_t rounds = 0;
        for (uint64_t w = kSortTile; w < a.m; w *= 2) ++rounds;
        uint64_t *buf[2] = {a.tkeys, a.tkeys_sorted};
        uint32_t cur = (rounds & 1) ? 0 : 1;
        hipLaunchKernelGGL(k_map_tile_sort, dim3((unsigned)((a.m + kSortTile - 1) / kSortTile)), dim3(256), 0, s, a,
                           a.tkeys, buf[cur]);
        const unsigned mblocks = blocks_for(std::min<uint64_t>(a.m, 1ull << 22));
        for (uint64_t w = kSortTile; w < a.m; w *= 2) {
            hipLaunchKernelGGL(k_map_merge, dim3(mblocks), dim3(256), 0, s, a, buf[cur], buf[cur ^ 1], w);
            cur ^= 1;
        }
        hipLaunchKernelGGL(k_map_zero, dim3(blocks_for(std::min<uint64_t>(a.m * 256, 1ull << 22))), dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL(k_map_write, dim3(blocks_for(std::max(a.n, a.m))), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace dv
