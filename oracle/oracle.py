"""ctypes binding of the C oracle (test infrastructure only).

The oracle owns nothing: the caller passes numpy byte arrays for each VM's
arena and for the host pool, and the oracle reads and writes them in place.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CODES = {
    "OK": 0, "NOT_PRESENT": 1, "RESERVED": 2, "PROT_USER": 3, "PROT_WRITE": 4,
    "NO_MEMSLOT": 5, "NONCANONICAL": 6, "INVALID": 7, "NO_POOL": 8, "EPT_VIOLATION": 9, "EPT_MISCONFIG": 10,
}
RESULT_DTYPE = np.dtype([("bytes_done", "<u8"), ("fault_gva", "<u8"), ("code", "<u4"), ("level", "<u2"),
                         ("pad", "<u2")])
FAULT_DTYPE = np.dtype([("req_index", "<u8"), ("fault_gva", "<u8"), ("code", "<u4"), ("level", "<u2"),
                        ("pad", "<u2")])
XLAT_DTYPE = np.dtype([("gpa", "<u8"), ("hpa", "<u8"), ("code", "<u4"), ("level", "u1"), ("page_shift", "u1"),
                       ("vm", "<u2")])
SLOT_DTYPE = np.dtype([("gpa", "<u8"), ("bytes", "<u8"), ("arena_off", "<u8")])
MAP_DTYPE = np.dtype([("gva", "<u8"), ("gpa", "<u8"), ("flags", "<u4"), ("pad", "<u4")])
EPT_MAP_DTYPE = np.dtype([("gpa", "<u8"), ("hpa", "<u8"), ("flags", "<u4"), ("pad", "<u4")])
XLAT_WRITE = 1
XLAT_SET_AD = 2


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-Wall", "-fPIC", "-shared", "-pthread", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_libs = {}


def _load(path: str | None = None):
    """Load the oracle library (``path`` lets a test load a deliberately broken build)."""
    key = path or _LIB
    if key not in _libs:
        if path is None and not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(key)
        vp, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        lib.orc_new.argtypes = [u32, u32]
        lib.orc_new.restype = vp
        lib.orc_free.argtypes = [vp]
        lib.orc_set_vm.argtypes = [vp, u32, vp, u64, vp, u32]
        lib.orc_set_proc.argtypes = [vp, u32, u32, u64, u32]
        lib.orc_set_ept.argtypes = [vp, u32, u64]
        lib.orc_set_ept.restype = ctypes.c_int
        lib.orc_set_pool.argtypes = [vp, vp, u64]
        lib.orc_ad_sets.argtypes = [vp]
        lib.orc_ad_sets.restype = u64
        lib.orc_translate.argtypes = [vp, u32, vp, u64, u32, vp]
        lib.orc_copy.argtypes = [vp, vp, vp]
        lib.orc_copy.restype = ctypes.c_int
        lib.orc_batch.argtypes = [vp, vp, u64, vp, vp]
        lib.orc_batch.restype = ctypes.c_int64
        lib.orc_batch_results.argtypes = [vp, vp, u64, vp, vp]
        lib.orc_batch_results.restype = ctypes.c_int64
        lib.orc_batch_ad.argtypes = [vp, vp, u64, vp, vp]
        lib.orc_batch_ad.restype = ctypes.c_int64
        lib.orc_batch_mt.argtypes = [vp, vp, u64, vp, u32, u32, ctypes.c_int, vp, vp]
        lib.orc_batch_mt.restype = ctypes.c_int64
        lib.orc_fifo_reset.argtypes = [vp, u32]
        lib.orc_fifo_reset.restype = ctypes.c_int
        lib.orc_fifo_counts.argtypes = [vp, u32, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        lib.orc_check_conflicts.argtypes = [vp, vp, u64, vp, u32, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        lib.orc_check_conflicts.restype = ctypes.c_int
        lib.orc_map_pages.argtypes = [vp, u32, vp, u64, vp, u64, vp]
        lib.orc_map_pages.restype = ctypes.c_int64
        lib.orc_ept_map_pages.argtypes = [vp, u32, vp, u64, vp, u64, vp]
        lib.orc_ept_map_pages.restype = ctypes.c_int64
        lib.orc_ept_xlat.argtypes = [vp, u32, u64, u32, ctypes.POINTER(u64)]
        lib.orc_ept_xlat.restype = u32
        _libs[key] = lib
    return _libs[key]


class Oracle:
    """State = arenas (one uint8 array per VM), memslots, processes and a pool.

    ``asid`` values are positions in the process list given at construction.
    """

    def __init__(self, arenas, slots, procs, pool, lib_path: str | None = None, ept=None):
        """arenas: list of uint8 arrays; slots: list of SLOT_DTYPE arrays;
        procs: list of (vm, cr3, levels); pool: uint8 array; ept: per VM the
        arena offset of its EPT root, or None for memslot translation."""
        lib = _load(lib_path)
        self._lib = lib
        self.arenas = [np.ascontiguousarray(a) for a in arenas]
        for a, b in zip(arenas, self.arenas):
            assert a is b, "arenas must be C-contiguous uint8 arrays (the oracle writes them in place)"
        self.slots = [np.ascontiguousarray(np.asarray(s, dtype=SLOT_DTYPE)) for s in slots]
        self.procs = list(procs)
        self.pool = pool
        assert pool.dtype == np.uint8 and pool.flags.c_contiguous
        self._h = lib.orc_new(len(arenas), len(procs))
        for i, (a, s) in enumerate(zip(self.arenas, self.slots)):
            assert a.dtype == np.uint8
            lib.orc_set_vm(self._h, i, a.ctypes.data, a.size, s.ctypes.data, len(s))
        for i, (vm, cr3, levels) in enumerate(self.procs):
            lib.orc_set_proc(self._h, i, vm, cr3, levels)
        for i, root in enumerate(ept or []):
            if root is not None and lib.orc_set_ept(self._h, i, int(root)) != 0:
                raise ValueError(f"bad EPT root {root:#x} for VM {i}")
        lib.orc_set_pool(self._h, pool.ctypes.data, pool.size)

    @classmethod
    def from_workload(cls, wl, arenas=None, pool=None, lib_path: str | None = None):
        if arenas is None:
            arenas = [wl.arena_image(v) for v in range(len(wl.vms))]
        if pool is None:
            pool = wl.pool_image()
        return cls(arenas, [v.slots for v in wl.vms], [(p.vm, p.cr3, p.levels) for p in wl.procs], pool,
                   lib_path=lib_path, ept=[getattr(v, "ept_root", None) for v in wl.vms])

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.orc_free(self._h)
            self._h = None

    @property
    def ad_sets(self) -> int:
        return int(self._lib.orc_ad_sets(self._h))

    def translate(self, asid: int, gvas, flags: int = 0) -> np.ndarray:
        g = np.ascontiguousarray(np.asarray(gvas, dtype=np.uint64).reshape(-1))
        out = np.zeros(len(g), XLAT_DTYPE)
        self._lib.orc_translate(self._h, asid, g.ctypes.data, len(g), flags, out.ctypes.data)
        return out

    def copy(self, req) -> np.ndarray:
        r = np.ascontiguousarray(np.asarray(req).reshape(1))
        res = np.zeros(1, RESULT_DTYPE)
        rc = self._lib.orc_copy(self._h, r.ctypes.data, res.ctypes.data)
        if rc != 0:
            raise ValueError("request names pool bytes outside the pool")
        return res[0]

    def batch(self, reqs):
        r = np.ascontiguousarray(reqs)
        n = len(r)
        res = np.zeros(n, RESULT_DTYPE)
        faults = np.zeros(n, FAULT_DTYPE)
        nf = self._lib.orc_batch(self._h, r.ctypes.data, n, res.ctypes.data, faults.ctypes.data)
        if nf < 0:
            raise ValueError("request names pool bytes outside the pool")
        return res, faults[:nf].copy()

    def batch_ad(self, reqs):
        """Results, fault list and A/D updates, without moving payload bytes."""
        r = np.ascontiguousarray(reqs)
        n = len(r)
        res = np.zeros(n, RESULT_DTYPE)
        faults = np.zeros(n, FAULT_DTYPE)
        nf = self._lib.orc_batch_ad(self._h, r.ctypes.data, n, res.ctypes.data, faults.ctypes.data)
        return res, faults[:nf].copy()

    def batch_mt(self, reqs, epoch_end=None, threads: int = 1, ad_only: bool = False):
        """The batch with each epoch's requests split over `threads` threads
        (the batch precondition makes that equal to the sequential batch);
        ad_only: A/D updates without payload moves, as batch_ad."""
        r = np.ascontiguousarray(reqs)
        n = len(r)
        e = np.ascontiguousarray(np.asarray(epoch_end if epoch_end is not None else [n], np.uint64))
        if len(e) == 0 or int(e[-1]) != n or np.any(np.diff(e.astype(np.int64)) < 0):
            raise ValueError("epoch ends must ascend and end at n")
        res = np.zeros(n, RESULT_DTYPE)
        faults = np.zeros(n, FAULT_DTYPE)
        nf = self._lib.orc_batch_mt(self._h, r.ctypes.data, n, e.ctypes.data, len(e), int(threads),
                                    2 if ad_only else 1, res.ctypes.data, faults.ctypes.data)
        if nf == -4:
            raise ValueError("the threaded batch is not defined with the translation cache on")
        if nf < 0:
            raise ValueError("request names pool bytes outside the pool")
        return res, faults[:nf].copy()

    def fifo_reset(self, entries: int = 10):
        """Turn the per-process translation cache on with `entries` slots (0: off) and empty it."""
        if self._lib.orc_fifo_reset(self._h, entries) != 0:
            raise ValueError("entries must be <= 64")

    def fifo_counts(self, asid: int):
        """(hits, misses) of a process's translation cache since the last reset."""
        h, m = ctypes.c_uint64(), ctypes.c_uint64()
        self._lib.orc_fifo_counts(self._h, asid, ctypes.byref(h), ctypes.byref(m))
        return int(h.value), int(m.value)

    def batch_results(self, reqs):
        """Results and fault list only (no byte moves, no A/D updates)."""
        r = np.ascontiguousarray(reqs)
        n = len(r)
        res = np.zeros(n, RESULT_DTYPE)
        faults = np.zeros(n, FAULT_DTYPE)
        nf = self._lib.orc_batch_results(self._h, r.ctypes.data, n, res.ctypes.data, faults.ctypes.data)
        return res, faults[:nf].copy()

    def map_pages(self, asid: int, maps, pool_gpa):
        """Map pages by writing the guest tables (see orc_map_pages); returns
        (per-map results, pool frames used)."""
        m = np.ascontiguousarray(maps, dtype=MAP_DTYPE)
        pool = np.ascontiguousarray(np.asarray(pool_gpa, np.uint64).reshape(-1))
        res = np.zeros(len(m), RESULT_DTYPE)
        used = self._lib.orc_map_pages(self._h, asid, m.ctypes.data, len(m), pool.ctypes.data if len(pool) else None,
                                       len(pool), res.ctypes.data)
        if used < 0:
            raise ValueError("a pool frame is unaligned or outside every memslot")
        return res, int(used)

    def ept_map_pages(self, vm: int, maps, pool_off):
        """Map guest-physical pages by writing VM vm's EPT (see orc_ept_map_pages);
        returns (per-map results, pool pages used)."""
        m = np.ascontiguousarray(maps, dtype=EPT_MAP_DTYPE)
        pool = np.ascontiguousarray(np.asarray(pool_off, np.uint64).reshape(-1))
        res = np.zeros(len(m), RESULT_DTYPE)
        used = self._lib.orc_ept_map_pages(self._h, vm, m.ctypes.data, len(m),
                                           pool.ctypes.data if len(pool) else None, len(pool), res.ctypes.data)
        if used < 0:
            raise ValueError("the VM has no EPT, or a pool page is unaligned, outside the arena or repeated")
        return res, int(used)

    def ept_xlat(self, vm: int, gpa: int, need: int = 0):
        """(code, arena offset) of gpa through VM vm's EPT; need: bit 0 read, bit 1 write."""
        h = ctypes.c_uint64()
        code = self._lib.orc_ept_xlat(self._h, vm, gpa, need, ctypes.byref(h))
        return int(code), int(h.value)

    def check_conflicts(self, reqs, epoch_end=None):
        """Return None if every epoch is conflict-free, else the offending (i, j)."""
        r = np.ascontiguousarray(reqs)
        e = np.ascontiguousarray(np.asarray(epoch_end if epoch_end is not None else [len(r)], np.uint64))
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        rc = self._lib.orc_check_conflicts(self._h, r.ctypes.data, len(r), e.ctypes.data, len(e),
                                           ctypes.byref(a), ctypes.byref(b))
        if rc < 0:
            raise MemoryError
        return None if rc == 0 else (int(a.value), int(b.value))
