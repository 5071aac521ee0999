"""Seeded generator for guest page tables, memslots, arenas and requests.

Workload recipe (each VM, each process):

* Guest-physical memory of ``mem_bytes`` is split into ``n_slots`` memslots at
  distinct uniformly drawn 4 KiB cut points.  The slots are laid out in the
  VM's arena in a random order, each preceded by a guard gap of 0-64 KiB that
  no slot maps, so a guest page that is contiguous in GPA need not be
  contiguous in the arena (the per-page translation of the software hybrid
  address space, section 4.2).
* Each process maps ``mapped_frac * mem_bytes / procs_per_vm`` bytes of user
  virtual address space, split by mapped bytes into 4 KiB, 2 MiB and 1 GiB
  leaves.  The space is built from 1 GiB blocks (one 1 GiB leaf), 2 MiB
  blocks (one 2 MiB leaf) and page-table blocks (up to 512 4 KiB leaves),
  shuffled and grouped into ``vmas_per_proc`` VMAs of near-equal size at
  random 1 GiB-aligned user addresses.
* Data frames are a random permutation of free GPA frames of the right
  alignment (1 GiB first, then 2 MiB, then 4 KiB); page-table frames are
  random free 4 KiB frames.  Leaves are not-present with probability
  ``p_np`` and then hold random bits with bit 0 clear.  Present entries carry
  random ignored bits and have A = D = 0.
* Requests pick a process uniformly, a direction by a Bernoulli draw and a
  length from the configured distribution.  They are cut into epochs greedily
  so that no epoch places more than ``rho`` of any VMA, and inside an epoch
  they are packed into their VMA in index order at random gaps, so requests
  of one epoch never overlap in guest memory.  Host offsets are disjoint
  within an epoch with a random 0-63 byte skew.  With ``pool_mode="unique"``
  every request has pool bytes of its own; with ``"reuse"`` each VM owns a
  range of the pool, and in every epoch its requests take consecutive
  stretches of that range from its start, so later epochs reuse the bytes of
  earlier ones while different VMs never share a pool byte.

The page-table format written here is the x86-64 one (4-level, and 5-level
with 57-bit addresses): 512 eight-byte entries per 4 KiB table; bit 0 present,
bit 1 writable, bit 2 user, bit 5 accessed, bit 6 dirty, bit 7 page size,
address bits 51:12.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

KiB = 1 << 10
MiB = 1 << 20
GiB = 1 << 30
PAGE = 4096

REQ_DTYPE = np.dtype([
    ("gva", "<u8"), ("host", "<u8"), ("len", "<u4"), ("asid", "<u4"),
    ("dir", "u1"), ("rsvd", "u1", (3,)), ("tag", "<u4"),
])
assert REQ_DTYPE.itemsize == 32
SLOT_DTYPE = np.dtype([("gpa", "<u8"), ("bytes", "<u8"), ("arena_off", "<u8")])

FROM_GUEST = 0
TO_GUEST = 1

# entry bits
_P, _RW, _US, _PS = 1, 2, 4, 0x80
_HI_IGN = np.uint64(((1 << 64) - 1) ^ ((1 << 52) - 1))        # bits 63:52
_IGN_PTE = np.uint64(0x0F98) | _HI_IGN    # PWT PCD PAT G AVL(11:9)
_IGN_LARGE = np.uint64(0x1F18) | _HI_IGN  # PWT PCD G AVL PAT(12)
_IGN_TABLE = np.uint64(0x0F18) | _HI_IGN  # PWT PCD G AVL
_ADDR = np.uint64(0x000FFFFFFFFFF000)
# PAE (levels 3): bits 62:52 are reserved in every entry, XD (63) is accepted;
# a page-directory-pointer entry has only P, PWT, PCD and the AVL bits 11:9
_XD = np.uint64(1 << 63)
_IGN_PTE_PAE = np.uint64(0x0F98) | _XD
_IGN_LARGE_PAE = np.uint64(0x1F18) | _XD
_IGN_TABLE_PAE = np.uint64(0x0F18) | _XD
_IGN_PDPTE = np.uint64(0x0E18)

POOL_KEY = 0xFFFF


# ---------------------------------------------------------------------------
# native helper (closed-form fill, epoch cut)
# ---------------------------------------------------------------------------
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libwlhelp.so")
_lib = None


def build_helper(force: bool = False) -> str:
    src = os.path.join(_HERE, "wlhelp.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", src, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _helper():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_helper()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.wl_fill.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                ctypes.c_uint64, ctypes.c_int]
        lib.wl_fill.restype = ctypes.c_int
        lib.wl_assign_epochs.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                         ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
        lib.wl_assign_epochs.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def _nthreads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def fill_bytes(out: np.ndarray, seed: int, key: int, off: int = 0) -> np.ndarray:
    """Write the closed-form fill bytes for absolute offsets [off, off+len(out))."""
    assert out.dtype == np.uint8 and out.flags.c_contiguous
    _helper().wl_fill(out.ctypes.data, off, out.size, seed & (2**64 - 1), key, _nthreads())
    return out


# ---------------------------------------------------------------------------
# configuration
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class Spec:
    name: str
    n_vms: int
    procs_per_vm: int
    mem_bytes: int
    levels: int
    mix: tuple            # (4 KiB, 2 MiB, 1 GiB) share of mapped bytes
    n_slots: int
    p_np: float
    n_requests: int
    len_kind: str         # "uniform" | "loguniform"
    len_lo: int
    len_hi: int
    seed: int
    p_to_guest: float = 0.5
    rho: float = 0.5
    pool_mode: str = "unique"   # "unique" buffers per request, or "reuse" per epoch
    mix_fleetwide: bool = False
    vmas_per_proc: int = 4
    mapped_frac: float = 0.5
    # fault-injection knobs used by tests (0 in the named configurations)
    p_readonly: float = 0.0     # present leaves with R/W = 0
    p_supervisor: float = 0.0   # present leaves with U/S = 0
    p_upper_np: float = 0.0     # upper-level (non-leaf) entries not present
    # a 4-level EPT for the guest-physical space (instead of memslot translation)
    ept: bool = False
    ept_align: int = 2 * MiB    # slots are placed in the arena congruent to their GPA modulo this
    ept_np: float = 0.0         # EPT leaves not present
    ept_ro: float = 0.0         # EPT leaves read-only
    ept_mis: float = 0.0        # EPT leaves misconfigured (write without read, or memory type 2)

    def replace(self, **kw) -> "Spec":
        return dataclasses.replace(self, **kw)


SPECS = {
    # one guest, 64 MiB, 8192 4 KiB pages, 10% not present, 256 requests 8-4096 B
    "C1": Spec("C1", 1, 1, 64 * MiB, 4, (1.0, 0.0, 0.0), 4, 0.10, 256, "uniform", 8, 4096, 1001),
    # one guest, 4 GiB, 70/30 4K/2M, 16 slots, 5% not present, 1e6 requests 64 B-64 KiB
    "C2": Spec("C2", 1, 1, 4 * GiB, 4, (0.7, 0.3, 0.0), 16, 0.05, 1_000_000, "loguniform", 64, 64 * KiB, 1002),
    # 16 VMs x 4 processes, 2 GiB each, 80/20, 4e6 requests 16 B-4 MiB
    "C3": Spec("C3", 16, 4, 2 * GiB, 4, (0.8, 0.2, 0.0), 8, 0.05, 4_000_000, "loguniform", 16, 4 * MiB, 1003,
               pool_mode="reuse"),
    # serving: 8 VMs x 4 processes of 4 GiB (requests come from the serving trace generator)
    "C4": Spec("C4", 8, 4, 4 * GiB, 4, (0.7, 0.3, 0.0), 16, 0.05, 0, "loguniform", 24, 4147200, 1004,
               pool_mode="reuse"),
    # 64 VMs x 2 GiB, 5-level paging, 60/35/5 (1 GiB share fleet-wide), 3% not present,
    # 1e7 requests 16 B-1 MiB
    "C5": Spec("C5", 64, 1, 2 * GiB, 5, (0.60, 0.35, 0.05), 8, 0.03, 10_000_000, "loguniform", 16, 1 * MiB, 1005,
               pool_mode="reuse", mix_fleetwide=True),
}


def spec(name: str, **kw) -> Spec:
    return SPECS[name].replace(**kw) if kw else SPECS[name]


# ---------------------------------------------------------------------------
# workload container
# ---------------------------------------------------------------------------
@dataclass
class VMImage:
    vm: int
    mem_bytes: int
    slots: np.ndarray           # SLOT_DTYPE, sorted by gpa
    arena_bytes: int
    pt_gfn: np.ndarray          # uint64 GPA frame numbers of page-table frames
    pt_data: np.ndarray         # (n, 512) uint64 table contents
    key: int
    ept_root: int | None = None     # arena offset of the EPT's level-4 table
    ept_off: np.ndarray | None = None   # arena offsets of the EPT table frames
    ept_data: np.ndarray | None = None  # (n, 512) uint64 EPT table contents
    ept_leaf: np.ndarray | None = None  # the EPT leaves as generated: gpa, shift, kind (EPT_LEAF_*)


@dataclass
class ProcTruth:
    """Ground-truth map a process's tables were encoded from."""
    asid: int
    vm: int
    levels: int
    cr3: int
    leaf_va: np.ndarray         # uint64 virtual address of each leaf
    leaf_level: np.ndarray      # uint8: 1 (4 KiB), 2 (2 MiB), 3 (1 GiB)
    leaf_frame: np.ndarray      # uint64 frame GPA (meaningful when present)
    leaf_present: np.ndarray    # bool
    leaf_entry: np.ndarray      # uint64 entry value as written
    leaf_table_gfn: np.ndarray  # uint64 frame holding the entry
    leaf_index: np.ndarray      # uint16 entry index in that frame
    tables: dict                # level -> (ids uint64, gfns uint64); id = va >> (12 + 9*level)
    vmas: np.ndarray            # (k, 2) uint64 [base, size)


@dataclass
class Workload:
    spec: Spec
    vms: list
    procs: list                 # ProcTruth, index == asid
    requests: np.ndarray        # REQ_DTYPE, host = offset into the pool
    epoch_end: np.ndarray       # uint64, ascending, last == n
    pool_bytes: int
    seed: int
    req_vma: np.ndarray = field(default=None)
    # reuse mode: VM v's requests use pool bytes [pool_vm[v, 0], pool_vm[v, 0] + pool_vm[v, 1])
    pool_vm: np.ndarray = field(default=None)

    # -- images -------------------------------------------------------------
    def arena_image(self, vm: int, out: np.ndarray | None = None) -> np.ndarray:
        v = self.vms[vm]
        if out is None:
            out = np.empty(v.arena_bytes, np.uint8)
        fill_bytes(out, self.seed, v.key)
        self.overlay_tables(vm, out)
        if v.ept_root is not None:
            out.reshape(-1, PAGE)[(v.ept_off >> np.uint64(12)).astype(np.int64)] = \
                v.ept_data.view(np.uint8).reshape(-1, PAGE)
        return out

    def overlay_tables(self, vm: int, arena: np.ndarray) -> None:
        v = self.vms[vm]
        if len(v.pt_gfn) == 0:
            return
        hpa = gpa_to_arena(v.slots, v.pt_gfn << np.uint64(12))
        assert np.all(hpa >= 0)
        pages = arena.reshape(-1, PAGE)
        pages[(hpa >> 12).astype(np.int64)] = v.pt_data.view(np.uint8).reshape(-1, PAGE)

    def pool_image(self, out: np.ndarray | None = None) -> np.ndarray:
        if out is None:
            out = np.empty(self.pool_bytes, np.uint8)
        return fill_bytes(out, self.seed, POOL_KEY)

    def requests_at(self, pool_base: int) -> np.ndarray:
        r = self.requests.copy()
        r["host"] += np.uint64(pool_base)
        return r

    @property
    def n_requests(self) -> int:
        return len(self.requests)

    def epochs(self):
        s = 0
        for e in self.epoch_end:
            yield s, int(e)
            s = int(e)


def workload_key(wl: Workload, name: str) -> str:
    """A name for the batch's shape: the workload's name and a digest of its
    spec, requests and epoch cuts (keys the tuning cache)."""
    import hashlib
    h = hashlib.blake2b(digest_size=8)
    h.update(repr(wl.spec).encode())
    h.update(np.ascontiguousarray(wl.requests).view(np.uint8).tobytes())
    h.update(np.ascontiguousarray(wl.epoch_end, np.uint64).tobytes())
    return f"{name}-{h.hexdigest()}"


def gpa_to_arena(slots: np.ndarray, gpa: np.ndarray) -> np.ndarray:
    """Place GPAs in the arena through the slot list (generator-side layout helper).

    Returns int64 arena offsets, -1 where no slot covers the address."""
    gpa = np.asarray(gpa, np.uint64)
    base = slots["gpa"]
    i = np.searchsorted(base, gpa, side="right").astype(np.int64) - 1
    ok = i >= 0
    ic = np.where(ok, i, 0)
    ok &= gpa < base[ic] + slots["bytes"][ic]
    off = (gpa - base[ic] + slots["arena_off"][ic]).astype(np.int64)
    return np.where(ok, off, -1)


# ---------------------------------------------------------------------------
# generation
# ---------------------------------------------------------------------------
def _memslots(rng, mem_bytes: int, n_slots: int, align: int = 0):
    nfr = mem_bytes // PAGE
    n_slots = max(1, min(n_slots, nfr))
    cuts = np.sort(rng.choice(np.arange(1, nfr, dtype=np.int64), n_slots - 1, replace=False)) if n_slots > 1 else \
        np.zeros(0, np.int64)
    bounds = np.concatenate([[0], cuts, [nfr]]).astype(np.uint64)
    gpa = bounds[:-1] << np.uint64(12)
    size = (bounds[1:] - bounds[:-1]) << np.uint64(12)
    order = rng.permutation(n_slots)
    gaps = rng.integers(0, 17, n_slots + 1).astype(np.uint64) * np.uint64(PAGE)  # 0-64 KiB
    arena_off = np.zeros(n_slots, np.uint64)
    pos = np.uint64(0)
    for k, s in enumerate(order):
        if align:  # congruent to the GPA modulo `align`, so large EPT leaves can map the slot
            pos += np.uint64((int(gpa[s]) - int(pos)) % align)
        else:
            pos += gaps[k]
        arena_off[s] = pos
        pos += size[s]
    arena_bytes = int(pos + gaps[-1])
    slots = np.zeros(n_slots, SLOT_DTYPE)
    slots["gpa"], slots["bytes"], slots["arena_off"] = gpa, size, arena_off
    return slots, arena_bytes


def _split_counts(sp: Spec):
    """Per-process (n_1g, n_2m, n_4k) leaf counts for every process of the fleet."""
    nproc = sp.n_vms * sp.procs_per_vm
    v_pages = int(sp.mapped_frac * sp.mem_bytes) // PAGE // sp.procs_per_vm
    f4, f2, f1 = sp.mix
    P1, P2 = GiB // PAGE, 2 * MiB // PAGE
    n1 = np.zeros(nproc, np.int64)
    n2 = np.zeros(nproc, np.int64)
    if sp.mix_fleetwide:
        total = v_pages * nproc
        want1 = int(round(f1 * total / P1))
        cap1 = v_pages // P1
        # deterministic: spread the 1 GiB leaves over evenly spaced processes
        if want1 and cap1:
            step = max(1, nproc // want1)
            for j in range(want1):
                n1[(j * step) % nproc] += 1
            n1 = np.minimum(n1, cap1)
        rest = v_pages - n1 * P1
        want2 = f2 * total / P2
        n2 = np.floor(want2 * rest / max(1, rest.sum()) + 0.5).astype(np.int64)
        n2 = np.minimum(n2, rest // P2)
    else:
        n1[:] = int(round(f1 * v_pages / P1))
        n2[:] = int(round(f2 * v_pages / P2))
        over = n1 * P1 + n2 * P2 > v_pages
        n2 = np.where(over, (v_pages - n1 * P1) // P2, n2)
    n4 = v_pages - n1 * P1 - n2 * P2
    return n1, n2, n4


def _layout_process(rng, sp: Spec, n1: int, n2: int, n4: int):
    """Virtual layout: returns leaves (va, level) and VMAs."""
    nblk4 = (n4 + 511) // 512
    kinds = np.concatenate([np.full(n2, 2, np.int8), np.full(nblk4, 1, np.int8)])
    rng.shuffle(kinds)
    # PTE counts per 4K block: all 512 except the last block
    blk_ptes = np.full(nblk4, 512, np.int64)
    if nblk4:
        blk_ptes[-1] = n4 - 512 * (nblk4 - 1)
    nb = len(kinds)
    k = max(1, min(sp.vmas_per_proc, nb + n1))
    # split the 2 MiB-block sequence into k contiguous groups of near-equal size
    # (each cut jittered by up to 20% of a group), so no VMA starves an epoch
    if nb > 1 and k > 1:
        even = np.arange(1, k) * nb / k
        jitter = (rng.random(k - 1) - 0.5) * 0.4 * nb / k
        cuts = np.unique(np.clip(np.round(even + jitter), 1, nb - 1).astype(np.int64))
    else:
        cuts = np.zeros(0, np.int64)
    groups = np.split(np.arange(nb), cuts) if nb else [np.zeros(0, np.int64)]
    while len(groups) < k:
        groups.append(np.zeros(0, np.int64))
    g1 = rng.integers(0, k, n1) if n1 else np.zeros(0, np.int64)
    sizes = np.array([int((g1 == j).sum()) * GiB + len(groups[j]) * 2 * MiB for j in range(k)], np.int64)
    if sp.levels == 3:
        # PAE: 32-bit addresses; VMAs in [4 MiB, 3 GiB), cells of whole 2 MiB units
        if n1:
            raise ValueError("PAE paging has no 1 GiB pages")
        unit = 2 * MiB
        span = int(max(1, -(-int(sizes.max()) // unit)))
        ncell = (3 * GiB - 4 * MiB) // ((span + 1) * unit)
        cells = rng.choice(ncell, k, replace=False)
        bases = np.uint64(4 * MiB) + cells.astype(np.uint64) * np.uint64((span + 1) * unit)
    else:
        span = int(max(1, -(-int(sizes.max()) // GiB)))  # in GiB
        limit = 1 << (47 if sp.levels == 4 else 56)
        ncell = (limit - 2 * GiB) // ((span + 1) * GiB)
        cells = rng.choice(ncell, k, replace=False)
        bases = np.uint64(GiB) + cells.astype(np.uint64) * np.uint64((span + 1) * GiB)
    va_l, lvl_l = [], []
    blk4_idx = np.cumsum(kinds == 1) - 1
    vmas = []
    for j in range(k):
        base = int(bases[j])
        pos = base
        for _ in range(int((g1 == j).sum())):
            va_l.append(np.array([pos], np.uint64))
            lvl_l.append(np.array([3], np.uint8))
            pos += GiB
        for b in groups[j]:
            if kinds[b] == 2:
                va_l.append(np.array([pos], np.uint64))
                lvl_l.append(np.array([2], np.uint8))
            else:
                cnt = int(blk_ptes[blk4_idx[b]])
                va_l.append(np.uint64(pos) + np.arange(cnt, dtype=np.uint64) * np.uint64(PAGE))
                lvl_l.append(np.full(cnt, 1, np.uint8))
            pos += 2 * MiB
        if pos > base:
            vmas.append((base, pos - base))
    va = np.concatenate(va_l) if va_l else np.zeros(0, np.uint64)
    lvl = np.concatenate(lvl_l) if lvl_l else np.zeros(0, np.uint8)
    return va, lvl, np.array(vmas, np.uint64).reshape(-1, 2)


_EPT_RWX, _EPT_WB = 7, 6 << 3
EPT_LEAF_OK, EPT_LEAF_NP, EPT_LEAF_RO, EPT_LEAF_MIS = 0, 1, 2, 3
EPT_LEAF_DTYPE = np.dtype([("gpa", "<u8"), ("shift", "u1"), ("kind", "u1")])


def _make_ept(rng, sp: Spec, slots: np.ndarray, arena_bytes: int):
    """A 4-level EPT mapping every slot's GPAs to the slot's arena bytes, with
    the largest leaf (1 GiB, 2 MiB, 4 KiB) that both sides' alignment allows;
    its tables are placed after the guest memory.  Returns (root, offsets,
    contents, new arena size)."""
    g_l, h_l, lv_l = [], [], []
    for sl in slots:
        g, end, h = int(sl["gpa"]), int(sl["gpa"] + sl["bytes"]), int(sl["arena_off"])
        while g < end:
            for lv, size in ((3, GiB), (2, 2 * MiB), (1, PAGE)):
                if g % size == 0 and h % size == 0 and g + size <= end:
                    break
            if lv == 1:  # a run of 4 KiB leaves up to the next 2 MiB boundary (or the slot end)
                stop = min(end, (g // (2 * MiB) + 1) * 2 * MiB)
                n = (stop - g) // PAGE
                g_l.append(np.uint64(g) + (np.arange(n, dtype=np.uint64) << np.uint64(12)))
                h_l.append(np.uint64(h) + (np.arange(n, dtype=np.uint64) << np.uint64(12)))
                lv_l.append(np.ones(n, np.uint8))
                g, h = stop, h + (stop - g)
            else:
                g_l.append(np.array([g], np.uint64))
                h_l.append(np.array([h], np.uint64))
                lv_l.append(np.array([lv], np.uint8))
                g, h = g + size, h + size
    lg, lh, ll = np.concatenate(g_l), np.concatenate(h_l), np.concatenate(lv_l)
    # tables: level L holds entries for gpa >> (12 + 9 (L-1)); its id is gpa >> (12 + 9 L)
    ids = {4: np.zeros(1, np.uint64)}
    need = {1: lg[ll == 1] >> np.uint64(21), 2: lg[ll <= 2] >> np.uint64(30), 3: lg >> np.uint64(39)}
    for L in (3, 2, 1):
        ids[L] = np.unique(need[L])
    n_tab = sum(len(ids[L]) for L in ids)
    base = (arena_bytes + PAGE - 1) // PAGE * PAGE
    off, o = {}, base
    for L in (4, 3, 2, 1):
        off[L] = np.uint64(o) + (np.arange(len(ids[L]), dtype=np.uint64) << np.uint64(12))
        o += len(ids[L]) * PAGE
    data = {L: np.zeros((len(ids[L]), 512), np.uint64) for L in ids}
    for L in (3, 2, 1):  # link tables at level L from level L+1
        parent = np.searchsorted(ids[L + 1], ids[L] >> np.uint64(9))
        data[L + 1][parent, (ids[L] & np.uint64(511)).astype(np.int64)] = off[L] | np.uint64(_EPT_RWX)
    ent = lh | np.uint64(_EPT_RWX | _EPT_WB) | np.where(ll > 1, np.uint64(0x80), np.uint64(0))
    r = rng.random(len(ent))
    truth = np.zeros(len(ent), EPT_LEAF_DTYPE)
    truth["gpa"], truth["shift"] = lg, (12 + 9 * (ll.astype(np.int64) - 1)).astype(np.uint8)
    truth["kind"] = np.select([r < sp.ept_np, r < sp.ept_np + sp.ept_ro, r < sp.ept_np + sp.ept_ro + sp.ept_mis],
                              [EPT_LEAF_NP, EPT_LEAF_RO, EPT_LEAF_MIS], EPT_LEAF_OK)
    ent = np.where(r < sp.ept_np, np.uint64(0), ent)
    ent = np.where((r >= sp.ept_np) & (r < sp.ept_np + sp.ept_ro), ent & ~np.uint64(2), ent)
    mis = (r >= sp.ept_np + sp.ept_ro) & (r < sp.ept_np + sp.ept_ro + sp.ept_mis)
    alt = rng.random(len(ent)) < 0.5
    ent = np.where(mis & alt, ent & ~np.uint64(1), ent)                                   # write without read
    ent = np.where(mis & ~alt, (ent & ~np.uint64(0x38)) | np.uint64(2 << 3), ent)         # memory type 2
    for L in (3, 2, 1):
        m = ll == L
        pos = np.searchsorted(ids[L], lg[m] >> np.uint64(12 + 9 * L))
        data[L][pos, ((lg[m] >> np.uint64(12 + 9 * (L - 1))) & np.uint64(511)).astype(np.int64)] = ent[m]
    offs = np.concatenate([off[L] for L in (4, 3, 2, 1)])
    cont = np.concatenate([data[L] for L in (4, 3, 2, 1)])
    order = np.argsort(truth["gpa"], kind="stable")
    return int(off[4][0]), offs, cont, o, truth[order]


def _rand_u64(rng, n):
    return rng.integers(0, 2**63, n, dtype=np.uint64) << np.uint64(1) | rng.integers(0, 2, n, dtype=np.uint64)


def make_workload(sp: Spec, requests: bool = True) -> Workload:
    rng = np.random.default_rng(sp.seed)
    nproc_vm = sp.procs_per_vm
    n1, n2, n4 = _split_counts(sp)
    vms, procs = [], []
    for vm in range(sp.n_vms):
        slots, arena_bytes = _memslots(rng, sp.mem_bytes, sp.n_slots, sp.ept_align if sp.ept else 0)
        nfr = sp.mem_bytes // PAGE
        free = np.ones(nfr, bool)
        lay = []
        for p in range(nproc_vm):
            a = vm * nproc_vm + p
            lay.append(_layout_process(rng, sp, int(n1[a]), int(n2[a]), int(n4[a])))
        # data frames: 1 GiB, then 2 MiB, then 4 KiB
        frames = []
        need = [(int(np.sum(l[1] == 3)), int(np.sum(l[1] == 2)), int(np.sum(l[1] == 1))) for l in lay]
        tot1, tot2, tot4 = (sum(x[i] for x in need) for i in range(3))
        P1, P2 = GiB // PAGE, 2 * MiB // PAGE
        c1 = rng.permutation(nfr // P1)[:tot1]
        for c in c1:
            free[c * P1:(c + 1) * P1] = False
        ok2 = free.reshape(-1, P2).all(axis=1) if nfr % P2 == 0 else \
            np.array([free[i * P2:(i + 1) * P2].all() for i in range(nfr // P2)])
        cand2 = np.nonzero(ok2)[0]
        if len(cand2) < tot2:
            raise ValueError("guest memory too small for the 2 MiB leaves")
        c2 = rng.permutation(cand2)[:tot2]
        for c in c2:
            free[c * P2:(c + 1) * P2] = False
        cand4 = np.nonzero(free)[0]
        if len(cand4) < tot4:
            raise ValueError("guest memory too small for the 4 KiB leaves")
        c4 = rng.permutation(cand4)[:tot4]
        free[c4] = False
        o1 = o2 = o4 = 0
        for p in range(nproc_vm):
            va, lvl, _ = lay[p]
            fr = np.zeros(len(va), np.uint64)
            m1, m2, m4 = lvl == 3, lvl == 2, lvl == 1
            fr[m1] = c1[o1:o1 + m1.sum()].astype(np.uint64) * np.uint64(GiB)
            fr[m2] = c2[o2:o2 + m2.sum()].astype(np.uint64) * np.uint64(2 * MiB)
            fr[m4] = c4[o4:o4 + m4.sum()].astype(np.uint64) * np.uint64(PAGE)
            o1 += int(m1.sum()); o2 += int(m2.sum()); o4 += int(m4.sum())
            frames.append(fr)
        # page-table frames: ids per level, then random free frames
        tbl_ids = []
        n_tables = 0
        for p in range(nproc_vm):
            va, lvl, _ = lay[p]
            per = {}
            for L in range(1, sp.levels + 1):
                sel = lvl <= L
                ids = np.unique(va[sel] >> np.uint64(12 + 9 * L)) if sel.any() else np.zeros(0, np.uint64)
                if L == sp.levels and len(ids) == 0:
                    ids = np.zeros(1, np.uint64)
                per[L] = ids
                n_tables += len(ids)
            tbl_ids.append(per)
        cand = np.nonzero(free)[0]
        if len(cand) < n_tables:
            raise ValueError("guest memory too small for the page tables")
        ptf = rng.permutation(cand)[:n_tables].astype(np.uint64)
        free[ptf.astype(np.int64)] = False
        pt_gfn_all, pt_data_all = [], []
        o = 0
        for p in range(nproc_vm):
            asid = vm * nproc_vm + p
            va, lvl, vmas = lay[p]
            per = tbl_ids[p]
            gfns = {}
            for L in range(1, sp.levels + 1):
                gfns[L] = ptf[o:o + len(per[L])]
                o += len(per[L])
            data = {L: np.zeros((len(per[L]), 512), np.uint64) for L in per}
            pae = sp.levels == 3
            # PAE: the 4-entry page-directory-pointer table sits at a random
            # 32-byte slot of its frame, which CR3 bits 11:5 name
            pdpt_slot = int(rng.integers(0, 128)) if pae else 0
            # upper-level entries: child table at level L-1 referenced from level L
            for L in range(2, sp.levels + 1):
                child = per[L - 1]
                if len(child) == 0:
                    continue
                parent_pos = np.searchsorted(per[L], child >> np.uint64(9))
                if pae and L == 3:
                    e = (gfns[L - 1] << np.uint64(12)) | np.uint64(_P) | (_rand_u64(rng, len(child)) & _IGN_PDPTE)
                else:
                    ign = _IGN_TABLE_PAE if pae else _IGN_TABLE
                    e = (gfns[L - 1] << np.uint64(12)) | np.uint64(_P | _RW | _US) | (_rand_u64(rng, len(child)) & ign)
                if sp.p_upper_np > 0:
                    np_m = rng.random(len(child)) < sp.p_upper_np
                    e = np.where(np_m, _rand_u64(rng, len(child)) & ~np.uint64(1), e)
                slot = (child & np.uint64(511)).astype(np.int64)
                if pae and L == 3:
                    slot = slot + 4 * pdpt_slot
                data[L][parent_pos, slot] = e
            # leaves
            n = len(va)
            present = rng.random(n) >= sp.p_np
            rnd = _rand_u64(rng, n)
            ent = np.where(lvl == 1, (frames[p] | np.uint64(_P | _RW | _US)) | (rnd & (_IGN_PTE_PAE if pae else _IGN_PTE)),
                           (frames[p] | np.uint64(_P | _RW | _US | _PS)) | (rnd & (_IGN_LARGE_PAE if pae else _IGN_LARGE)))
            if sp.p_readonly > 0:
                ro = rng.random(n) < sp.p_readonly
                ent = np.where(ro, ent & ~np.uint64(_RW), ent)
            if sp.p_supervisor > 0:
                sv = rng.random(n) < sp.p_supervisor
                ent = np.where(sv, ent & ~np.uint64(_US), ent)
            ent = np.where(present, ent, _rand_u64(rng, n) & ~np.uint64(1))
            t_gfn = np.zeros(n, np.uint64)
            t_idx = np.zeros(n, np.uint16)
            for L in (1, 2, 3):
                m = lvl == L
                if not m.any():
                    continue
                tid = va[m] >> np.uint64(12 + 9 * L)
                pos = np.searchsorted(per[L], tid)
                idx = ((va[m] >> np.uint64(12 + 9 * (L - 1))) & np.uint64(511)).astype(np.int64)
                data[L][pos, idx] = ent[m]
                t_gfn[m] = gfns[L][pos]
                t_idx[m] = idx
            for L in per:
                pt_gfn_all.append(gfns[L])
                pt_data_all.append(data[L])
            root = int(gfns[sp.levels][0])
            if pae:
                cr3 = (root << 12) | (pdpt_slot << 5) | int(rng.integers(0, 32))  # bits 4:0 ignored
            else:
                cr3 = (root << 12) | int(rng.integers(0, 4096))   # low 12 bits ignored by the walk
            procs.append(ProcTruth(asid, vm, sp.levels, cr3, va, lvl, frames[p], present, ent, t_gfn, t_idx,
                                   {L: (per[L], gfns[L]) for L in per}, vmas))
        img = VMImage(vm, sp.mem_bytes, slots, arena_bytes, np.concatenate(pt_gfn_all),
                      np.concatenate(pt_data_all), vm)
        if sp.ept:
            img.ept_root, img.ept_off, img.ept_data, img.arena_bytes, img.ept_leaf = _make_ept(rng, sp, slots,
                                                                                              arena_bytes)
        vms.append(img)
    wl = Workload(sp, vms, procs, np.zeros(0, REQ_DTYPE), np.zeros(0, np.uint64), 0, sp.seed)
    if requests and sp.n_requests > 0:
        _make_requests(rng, sp, wl)
    return wl


def draw_lengths(rng, kind: str, lo: int, hi: int, n: int) -> np.ndarray:
    if kind == "uniform":
        return rng.integers(lo, hi + 1, n).astype(np.uint64)
    if kind == "loguniform":
        u = rng.random(n)
        return np.minimum(hi, np.floor(lo * (hi / lo) ** u)).astype(np.uint64)
    raise ValueError(kind)


def _make_requests(rng, sp: Spec, wl: Workload) -> None:
    n = sp.n_requests
    nproc = len(wl.procs)
    asid = rng.integers(0, nproc, n).astype(np.uint32)
    direction = (rng.random(n) < sp.p_to_guest).astype(np.uint8)
    length = draw_lengths(rng, sp.len_kind, sp.len_lo, sp.len_hi, n)
    # global VMA table
    vma_base, vma_size, vma_first = [], [], []
    for p in wl.procs:
        vma_first.append(len(vma_base))
        for b, s in p.vmas:
            vma_base.append(int(b)); vma_size.append(int(s))
    vma_first.append(len(vma_base))
    vma_base = np.array(vma_base, np.uint64)
    vma_size = np.array(vma_size, np.uint64)
    vma_first = np.array(vma_first, np.int64)
    # VMA per request, proportional to VMA size within its process
    u = rng.random(n)
    vma = np.zeros(n, np.uint32)
    for a in range(nproc):
        m = asid == a
        if not m.any():
            continue
        s = vma_size[vma_first[a]:vma_first[a + 1]].astype(np.float64)
        cdf = np.cumsum(s) / s.sum()
        vma[m] = (vma_first[a] + np.minimum(np.searchsorted(cdf, u[m], side="right"), len(s) - 1)).astype(np.uint32)
    budget = np.floor(sp.rho * vma_size.astype(np.float64)).astype(np.uint64)
    length = np.minimum(length, budget[vma])
    length = np.maximum(length, 1)
    # epochs
    lib = _helper()
    used = np.zeros(len(vma_size), np.uint64)
    epoch_end = np.zeros(n + 1, np.uint64)
    ne = lib.wl_assign_epochs(vma.ctypes.data, length.ctypes.data, n, budget.ctypes.data, len(vma_size),
                              used.ctypes.data, epoch_end.ctypes.data)
    epoch_end = epoch_end[:ne].copy()
    epoch_of = np.repeat(np.arange(ne, dtype=np.int64), np.diff(np.concatenate([[0], epoch_end.astype(np.int64)])))
    # placement inside (epoch, vma) groups, in index order at random sorted gaps
    g = epoch_of * len(vma_size) + vma.astype(np.int64)
    by_g = np.argsort(g, kind="stable")
    gs = g[by_g]
    starts = np.concatenate([[0], np.nonzero(np.diff(gs))[0] + 1])
    counts = np.diff(np.concatenate([starts, [n]]))
    grp_len = np.add.reduceat(length[by_g], starts) if n else np.zeros(0, np.uint64)
    grp_vma = vma[by_g][starts].astype(np.int64)
    free = vma_size[grp_vma] - grp_len
    uu = rng.random(n)
    u_sorted = uu[np.lexsort((uu, g))]
    seg_id = np.repeat(np.arange(len(starts)), counts)
    t = np.floor(u_sorted * (free[seg_id].astype(np.float64) + 1.0)).astype(np.uint64)
    t = np.minimum(t, free[seg_id])     # sorted draws keep t non-decreasing inside a group
    lc = np.cumsum(length[by_g].astype(np.int64))
    excl = lc - length[by_g].astype(np.int64) - np.repeat(lc[starts] - length[by_g][starts].astype(np.int64), counts)
    gva = np.zeros(n, np.uint64)
    gva[by_g] = vma_base[vma[by_g]] + t.astype(np.uint64) + excl.astype(np.uint64)
    # host offsets
    skew = rng.integers(0, 64, n).astype(np.uint64)
    span = length + skew
    if sp.pool_mode == "unique":
        host = np.cumsum(span) - length
        pool = int(host[-1] + length[-1]) if n else 0
    else:
        # consecutive stretches per (epoch, VM), inside the VM's own pool range
        n_vms = len(wl.vms)
        vm_of = np.array([p.vm for p in wl.procs], np.int64)[asid] if n else np.zeros(0, np.int64)
        key = epoch_of * n_vms + vm_of
        order = np.argsort(key, kind="stable")
        ks = key[order]
        sp_o = span[order].astype(np.int64)
        cs = np.cumsum(sp_o)
        first = np.concatenate([[0], np.nonzero(np.diff(ks))[0] + 1]) if n else np.zeros(0, np.int64)
        gid = np.repeat(np.arange(len(first)), np.diff(np.concatenate([first, [n]])))
        end_in = cs - (cs[first] - sp_o[first])[gid]      # end of each request inside its stretch
        need = np.zeros(n_vms, np.int64)
        if n:
            np.maximum.at(need, vm_of[order[first]], end_in[np.concatenate([first[1:] - 1, [n - 1]])])
        size = (need + 4095) & ~4095
        vbase = np.concatenate([[0], np.cumsum(size)[:-1]]).astype(np.int64)
        host = np.zeros(n, np.uint64)
        host[order] = (vbase[vm_of[order]] + end_in - length[order].astype(np.int64)).astype(np.uint64)
        pool = int(size.sum())
        wl.pool_vm = np.stack([vbase, size], axis=1).astype(np.uint64)
    pool = (pool + 4095) & ~4095
    req = np.zeros(n, REQ_DTYPE)
    req["gva"], req["host"], req["len"], req["asid"], req["dir"] = gva, host, length.astype(np.uint32), asid, direction
    wl.requests = req
    wl.epoch_end = epoch_end
    wl.pool_bytes = pool
    wl.req_vma = vma


# ---------------------------------------------------------------------------
# locality traces (the per-process translation cache)
# ---------------------------------------------------------------------------
def make_locality_trace(wl: Workload, n_ops: int, hot_buffers: int = 4, p_hot: float = 0.95,
                        max_hot_len: int = 4 * KiB, cold_hi: int = 16 * KiB, seed: int | None = None):
    """Operations, one at a time per process, that revisit a few buffers: each
    process owns `hot_buffers` buffers of 16 B - max_hot_len at random places
    of its VMAs (a driver's command, status and staging buffers); an operation
    touches one of them with probability p_hot (a random stretch inside it),
    else a random place of the process's VMAs (log-uniform 16 B - cold_hi).
    Processes are uniform, directions Bernoulli(0.5); host bytes are unique
    per operation.  Returns (requests, pool_bytes)."""
    rng = np.random.default_rng(wl.seed * 11 + 3 if seed is None else seed)
    bufs = []
    for p in wl.procs:
        vm = p.vmas[rng.integers(0, len(p.vmas), hot_buffers)]
        blen = draw_lengths(rng, "loguniform", 16, max_hot_len, hot_buffers)
        off = (rng.random(hot_buffers) * (vm[:, 1] - blen).astype(np.float64)).astype(np.uint64)
        bufs.append(np.stack([vm[:, 0] + off, blen], axis=1))
    bufs = np.array(bufs, np.uint64)                       # (procs, hot, 2)
    asid = rng.integers(0, len(wl.procs), n_ops)
    hot = rng.random(n_ops) < p_hot
    which = rng.integers(0, hot_buffers, n_ops)
    b = bufs[asid, which]
    u = rng.random(n_ops)
    hlen = np.maximum(1, np.floor(b[:, 1].astype(np.float64) * np.maximum(u, 1e-3))).astype(np.uint64)
    hoff = (rng.random(n_ops) * (b[:, 1] - hlen + np.uint64(1)).astype(np.float64)).astype(np.uint64)
    clen = draw_lengths(rng, "loguniform", 16, cold_hi, n_ops)
    gva = np.zeros(n_ops, np.uint64)
    length = np.where(hot, hlen, clen).astype(np.uint64)
    for a, p in enumerate(wl.procs):
        m = (asid == a) & ~hot
        if not m.any():
            continue
        v = p.vmas[rng.integers(0, len(p.vmas), int(m.sum()))]
        ln = np.minimum(length[m], v[:, 1])
        length[m] = ln
        gva[m] = v[:, 0] + (rng.random(int(m.sum())) * (v[:, 1] - ln + np.uint64(1)).astype(np.float64)).astype(np.uint64)
    gva[hot] = b[hot, 0] + hoff[hot]
    host = np.cumsum(length + np.uint64(64)) - length
    req = np.zeros(n_ops, REQ_DTYPE)
    req["gva"], req["host"], req["len"] = gva, host, length.astype(np.uint32)
    req["asid"], req["dir"] = asid.astype(np.uint32), (rng.random(n_ops) < 0.5).astype(np.uint8)
    pool = int(host[-1] + length[-1]) if n_ops else 0
    return req, (pool + 4095) & ~4095


# ---------------------------------------------------------------------------
# serving traces
# ---------------------------------------------------------------------------
# Operation classes of the device classes the paper devirtualizes (input,
# audio, GPU, camera): (share, length kind, lo, hi, direction).
C4_CLASSES = (
    (0.60, "uniform", 24, 24, TO_GUEST),                     # 64-bit input events, read() into the guest
    (0.25, "uniform", 4096, 4096, FROM_GUEST),               # audio periods, write() from the guest
    (0.14, "loguniform", 16 * KiB, 256 * KiB, FROM_GUEST),   # GPU command buffers, ioctl() submit
    (0.01, "uniform", 4147200, 4147200, TO_GUEST),           # 1920x1080 YUYV camera frames, read()
)


@dataclass
class ServingTrace:
    requests: np.ndarray      # REQ_DTYPE; host = offset into the trace pool; tag = guest thread id
    arrival_ns: np.ndarray    # uint64, ascending, from 0
    pool_bytes: int
    windows: np.ndarray       # (threads, 3) uint64: asid, tag, window base
    rate_per_s: float


def make_serving_trace(wl: Workload, n_ops: int, rate_per_s: float, threads_per_proc: int = 64,
                       window: int = 6 * MiB, classes=C4_CLASSES, host_mode: str = "per_thread",
                       seed: int | None = None) -> ServingTrace:
    """Poisson arrivals of class-mixed operations from guest threads that each
    own a private window of mapped virtual memory (so operations of different
    threads never overlap, and one thread's operations run one at a time).

    host_mode "per_thread": each thread owns one host buffer of `window` bytes
    (enough for any of its operations, which never overlap in time);
    "unique": every operation gets its own host bytes."""
    rng = np.random.default_rng(wl.seed * 7 + 1 if seed is None else seed)
    wins = []
    for p in wl.procs:
        k = 0
        for b, s in p.vmas:
            for j in range(int(s) // window):
                if k < threads_per_proc:
                    wins.append((p.asid, k, int(b) + j * window))
                    k += 1
        if k < threads_per_proc:
            raise ValueError(f"process {p.asid} has room for {k} windows of {window} bytes, "
                             f"{threads_per_proc} needed")
    wins = np.array(wins, np.uint64)
    nt = len(wins)
    shares = np.array([c[0] for c in classes])
    cls = rng.choice(len(classes), n_ops, p=shares / shares.sum())
    length = np.zeros(n_ops, np.uint64)
    direction = np.zeros(n_ops, np.uint8)
    for i, (_, kind, lo, hi, d) in enumerate(classes):
        m = cls == i
        length[m] = np.minimum(draw_lengths(rng, kind, lo, hi, int(m.sum())), window)
        direction[m] = d
    th = rng.integers(0, nt, n_ops)
    off = (rng.random(n_ops) * (np.uint64(window) - length + np.uint64(1)).astype(np.float64)).astype(np.uint64)
    gva = wins[th, 2] + off
    if host_mode == "unique":
        skew = rng.integers(0, 64, n_ops).astype(np.uint64)
        host = np.cumsum(length + skew) - length
        pool = int(host[-1] + length[-1]) if n_ops else 0
    else:
        host = th.astype(np.uint64) * np.uint64(window) + rng.integers(0, 64, n_ops).astype(np.uint64)
        host = np.minimum(host, th.astype(np.uint64) * np.uint64(window) + np.uint64(window) - length)
        pool = nt * window
    gaps = rng.exponential(1e9 / rate_per_s, n_ops)
    arrival = np.cumsum(gaps).astype(np.uint64)
    req = np.zeros(n_ops, REQ_DTYPE)
    req["gva"], req["host"], req["len"] = gva, host, length.astype(np.uint32)
    req["asid"], req["dir"], req["tag"] = wins[th, 0].astype(np.uint32), direction, wins[th, 1].astype(np.uint32)
    return ServingTrace(req, arrival, (pool + 4095) & ~4095, wins, rate_per_s)
