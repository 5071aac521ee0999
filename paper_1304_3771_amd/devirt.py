"""ctypes binding of libdevirt.so (argument marshalling only).

Every function maps one-to-one onto a C entry point of include/devirt.h and
keeps its name.  Buffers may be given as integers (device or host addresses),
as torch tensors (their data_ptr()) or as numpy arrays (host).  Streams may
be torch streams, raw handles or None (the null stream).  Every step of the
data path runs in the library's HIP kernels; if the library is missing this
module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdevirt.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "devirt.h")

FROM_GUEST, TO_GUEST = 0, 1
XLAT_WRITE, XLAT_SET_AD = 1, 2
CODES = {"OK": 0, "NOT_PRESENT": 1, "RESERVED": 2, "PROT_USER": 3, "PROT_WRITE": 4, "NO_MEMSLOT": 5,
         "NONCANONICAL": 6, "INVALID": 7, "NO_POOL": 8,
         "EPT_VIOLATION": 9, "EPT_MISCONFIG": 10}

REQUEST_DTYPE = np.dtype([("gva", "<u8"), ("host", "<u8"), ("len", "<u4"), ("asid", "<u4"), ("dir", "u1"),
                          ("rsvd", "u1", (3,)), ("tag", "<u4")])
RESULT_DTYPE = np.dtype([("bytes_done", "<u8"), ("fault_gva", "<u8"), ("code", "<u4"), ("level", "<u2"),
                         ("pad", "<u2")])
FAULT_DTYPE = np.dtype([("req_index", "<u8"), ("fault_gva", "<u8"), ("code", "<u4"), ("level", "<u2"),
                        ("pad", "<u2")])
XLAT_DTYPE = np.dtype([("gpa", "<u8"), ("hpa", "<u8"), ("code", "<u4"), ("level", "u1"), ("page_shift", "u1"),
                       ("vm", "<u2")])
MAP_DTYPE = np.dtype([("gva", "<u8"), ("gpa", "<u8"), ("flags", "<u4"), ("pad", "<u4")])
MAP_WRITE = 1
EPT_MAP_DTYPE = np.dtype([("gpa", "<u8"), ("hpa", "<u8"), ("flags", "<u4"), ("pad", "<u4")])
EPT_R, EPT_W, EPT_X = 1, 2, 4


class DevirtError(RuntimeError):
    def __init__(self, fn: str, rc: int, msg: str):
        super().__init__(f"{fn} failed ({rc}): {msg}")
        self.rc = rc


PROF_TIMING, PROF_COUNTERS = 1, 2  # devirt_set_profiling flags
SERVE_MODES = {"poll": 0, "notify": 1, "blocking": 2}  # devirt_server_cfg.flags
SERVE_DEVICE_TIMES = 0x100


class Config(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in (
        "group", "seg_chunks", "xlat_wg", "xlat_wgs_per_cu", "copy_wg", "copy_wgs_per_cu", "nontemporal",
        "inline_bytes", "use_graph", "overlap", "fifo_entries", "large_pages", "spill_side")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_uint64), ("epochs", ctypes.c_uint64), ("plain_calls", ctypes.c_uint64),
                ("graph_replays", ctypes.c_uint64), ("copy_launches", ctypes.c_uint64), ("copy_ms", ctypes.c_double),
                ("xlat_launches", ctypes.c_uint64), ("xlat_ms", ctypes.c_double),
                ("pages_walked", ctypes.c_uint64), ("cache_hits", ctypes.c_uint64), ("cache_misses", ctypes.c_uint64),
                ("segments", ctypes.c_uint64), ("inline_segments", ctypes.c_uint64), ("ad_atomics", ctypes.c_uint64),
                ("spilled_groups", ctypes.c_uint64), ("large_requests", ctypes.c_uint64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class ServerCfg(ctypes.Structure):
    _fields_ = [("max_inflight", ctypes.c_uint32), ("pool_bytes", ctypes.c_uint64), ("max_batch", ctypes.c_uint32),
                ("streams", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "loops", "launches", "ops", "ns_inbox", "ns_complete", "ns_admit", "ns_launch", "direct_launches")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Result(ctypes.Structure):
    _fields_ = [("bytes_done", ctypes.c_uint64), ("fault_gva", ctypes.c_uint64), ("code", ctypes.c_uint32),
                ("level", ctypes.c_uint16), ("pad", ctypes.c_uint16)]


class Completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("res", Result), ("t_submit_ns", ctypes.c_uint64),
                ("t_admit_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64), ("dev_start_ns", ctypes.c_uint64),
                ("dev_end_ns", ctypes.c_uint64)]


COMPLETION_DTYPE = np.dtype([("ticket", "<u8"), ("bytes_done", "<u8"), ("fault_gva", "<u8"), ("code", "<u4"),
                             ("level", "<u2"), ("pad", "<u2"), ("t_submit_ns", "<u8"), ("t_admit_ns", "<u8"),
                             ("t_done_ns", "<u8"), ("dev_start_ns", "<u8"), ("dev_end_ns", "<u8")])
assert COMPLETION_DTYPE.itemsize == ctypes.sizeof(Completion)

_lib = None
vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
_SIGS = {
    "devirt_open": ([i32, ctypes.POINTER(vp)]),
    "devirt_close": ([vp]),
    "devirt_vm_create": ([vp, u64, ctypes.POINTER(u32)]),
    "devirt_vm_arena": ([vp, u32, ctypes.POINTER(vp), ctypes.POINTER(u64)]),
    "devirt_vm_write": ([vp, u32, u64, vp, u64]),
    "devirt_vm_read": ([vp, u32, u64, vp, u64]),
    "devirt_memslot_set": ([vp, u32, u32, u64, u64, u64]),
    "devirt_vm_set_ept": ([vp, u32, u64]),
    "devirt_process_create": ([vp, u32, u64, u32, ctypes.POINTER(u32)]),
    "devirt_translate": ([vp, u32, vp, u64, u32, vp, vp]),
    "devirt_copy_from_guest": ([vp, u32, u64, vp, u64, vp, vp]),
    "devirt_copy_to_guest": ([vp, u32, u64, vp, u64, vp, vp]),
    "devirt_copy_static": ([vp, u32, u64, vp, u64, u32, vp, vp]),
    "devirt_submit_batch": ([vp, vp, u64, vp, u32, vp, vp, vp, vp, vp]),
    "devirt_map_pages": ([vp, u32, vp, u64, vp, u64, vp, vp, vp]),
    "devirt_ept_map_pages": ([vp, u32, vp, u64, vp, u64, vp, vp, vp]),
    "devirt_sync": ([vp, vp]),
    "devirt_get_config": ([vp, ctypes.POINTER(Config)]),
    "devirt_set_config": ([vp, ctypes.POINTER(Config)]),
    "devirt_autotune": ([vp, vp, u64, vp, u32, vp, vp, vp, vp, u32, ctypes.POINTER(Config),
                         ctypes.POINTER(ctypes.c_double)]),
    "devirt_autotune_cached": ([vp, ctypes.c_char_p, ctypes.c_char_p, vp, u64, vp, u32, vp, vp, vp, vp, u32,
                                ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)]),
    "devirt_fifo_counts": ([vp, u32, ctypes.POINTER(u64), ctypes.POINTER(u64)]),
    "devirt_fifo_flush": ([vp]),
    "devirt_set_profiling": ([vp, i32]),
    "devirt_get_stats": ([vp, ctypes.POINTER(Stats)]),
    "devirt_reset_stats": ([vp]),
    "devirt_server_start": ([vp, ctypes.POINTER(ServerCfg), ctypes.POINTER(vp)]),
    "devirt_server_submit": ([vp, vp, u32, ctypes.POINTER(u32)]),
    "devirt_server_submit_map": ([vp, u32, u32, vp, u32, vp, u32, vp, ctypes.POINTER(u64)]),
    "devirt_server_submit_ept_map": ([vp, u32, u32, u32, vp, u32, vp, u32, vp, ctypes.POINTER(u64)]),
    "devirt_server_poll": ([vp, vp, u32, ctypes.POINTER(u32)]),
    "devirt_server_drain": ([vp]),
    "devirt_server_stop": ([vp]),
    "devirt_server_get_stats": ([vp, ctypes.POINTER(ServerStats)]),
}


def header_functions() -> list:
    """Names of the functions include/devirt.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(devirt_[a-z_0-9]+)\s*\(", txt)))


def lib():
    """Load libdevirt.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1304_3771_amd/build.py "
                               "(or __graft_entry__.build()) -- there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.devirt_last_error.argtypes = []
        L.devirt_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take a pointer of {type(x)}")


def _stream(s):
    if s is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except Exception:  # pragma: no cover
            pass
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _check(fn: str, rc: int):
    if rc != 0:
        msg = lib().devirt_last_error()
        raise DevirtError(fn, rc, msg.decode() if msg else "")


class Context:
    """One devirt context on one HIP device."""

    def __init__(self, device: int = 0):
        self._h = vp()
        _check("devirt_open", lib().devirt_open(device, ctypes.byref(self._h)))
        self.device = device

    def close(self):
        if self._h:
            _check("devirt_close", lib().devirt_close(self._h))
            self._h = vp()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---- guest memory and tables
    def vm_create(self, arena_bytes: int) -> int:
        v = u32()
        _check("devirt_vm_create", lib().devirt_vm_create(self._h, arena_bytes, ctypes.byref(v)))
        return v.value

    def vm_arena(self, vm: int):
        p, n = vp(), u64()
        _check("devirt_vm_arena", lib().devirt_vm_arena(self._h, vm, ctypes.byref(p), ctypes.byref(n)))
        return p.value, n.value

    def vm_write(self, vm: int, off: int, src, nbytes: int | None = None):
        if nbytes is None:
            nbytes = src.nbytes if isinstance(src, np.ndarray) else src.numel() * src.element_size()
        _check("devirt_vm_write", lib().devirt_vm_write(self._h, vm, off, _ptr(src), nbytes))

    def vm_read(self, vm: int, off: int, out, nbytes: int | None = None):
        if nbytes is None:
            nbytes = out.nbytes if isinstance(out, np.ndarray) else out.numel() * out.element_size()
        _check("devirt_vm_read", lib().devirt_vm_read(self._h, vm, off, _ptr(out), nbytes))
        return out

    def memslot_set(self, vm: int, slot: int, gpa: int, nbytes: int, arena_off: int):
        _check("devirt_memslot_set", lib().devirt_memslot_set(self._h, vm, slot, gpa, nbytes, arena_off))

    def vm_set_ept(self, vm: int, root: int | None):
        """Translate the VM's guest-physical addresses through the EPT rooted
        at arena offset `root` (None: back to the memslots)."""
        _check("devirt_vm_set_ept", lib().devirt_vm_set_ept(self._h, vm, (1 << 64) - 1 if root is None else root))

    def process_create(self, vm: int, cr3: int, levels: int) -> int:
        a = u32()
        _check("devirt_process_create", lib().devirt_process_create(self._h, vm, cr3, levels, ctypes.byref(a)))
        return a.value

    # ---- data path
    def translate(self, asid: int, gvas, n: int, flags: int, out, stream=None):
        _check("devirt_translate",
               lib().devirt_translate(self._h, asid, _ptr(gvas), n, flags, _ptr(out), _stream(stream)))

    def copy_from_guest(self, asid: int, gva: int, dst, nbytes: int, res, stream=None):
        _check("devirt_copy_from_guest", lib().devirt_copy_from_guest(self._h, asid, gva, _ptr(dst), nbytes,
                                                                      _ptr(res), _stream(stream)))

    def copy_to_guest(self, asid: int, gva: int, src, nbytes: int, res, stream=None):
        _check("devirt_copy_to_guest", lib().devirt_copy_to_guest(self._h, asid, gva, _ptr(src), nbytes,
                                                                  _ptr(res), _stream(stream)))

    def copy_static(self, asid: int, gva: int, host, nbytes: int, direction: int, res, stream=None):
        """The per-request copy with its scratch in a static device array (allocates nothing)."""
        _check("devirt_copy_static", lib().devirt_copy_static(self._h, asid, gva, _ptr(host), nbytes, direction,
                                                              _ptr(res), _stream(stream)))

    def map_pages(self, asid: int, maps, n: int, pool_gpa, res, n_used, stream=None):
        """maps: device array of MAP_DTYPE records; pool_gpa: host sequence of
        free guest frames; res: device results; n_used: device uint64."""
        pool = np.ascontiguousarray(np.asarray(pool_gpa, dtype=np.uint64).reshape(-1))
        _check("devirt_map_pages", lib().devirt_map_pages(
            self._h, asid, _ptr(maps), n, pool.ctypes.data if len(pool) else None, len(pool), _ptr(res),
            _ptr(n_used), _stream(stream)))

    def ept_map_pages(self, vm: int, maps, n: int, pool, res, n_used, stream=None):
        """maps: device array of EPT_MAP_DTYPE records; pool: host sequence of
        free arena pages (offsets); res: device results; n_used: device uint64."""
        pool = np.ascontiguousarray(np.asarray(pool, dtype=np.uint64).reshape(-1))
        _check("devirt_ept_map_pages", lib().devirt_ept_map_pages(
            self._h, vm, _ptr(maps), n, pool.ctypes.data if len(pool) else None, len(pool), _ptr(res),
            _ptr(n_used), _stream(stream)))

    def submit_batch(self, reqs, n: int, res, epoch_end=None, faults=None, n_faults=None, t_done=None,
                     stream=None):
        ep = None
        ne = 0
        if epoch_end is not None:
            ep = np.ascontiguousarray(np.asarray(epoch_end, dtype=np.uint64))
            ne = len(ep)
        _check("devirt_submit_batch", lib().devirt_submit_batch(
            self._h, _ptr(reqs), n, ep.ctypes.data if ep is not None else None, ne, _ptr(res), _ptr(faults),
            _ptr(n_faults), _ptr(t_done), _stream(stream)))

    def sync(self, stream=None):
        _check("devirt_sync", lib().devirt_sync(self._h, _stream(stream)))

    # ---- tuning and metrics
    def get_config(self) -> dict:
        c = Config()
        _check("devirt_get_config", lib().devirt_get_config(self._h, ctypes.byref(c)))
        return c.as_dict()

    def set_config(self, **kw):
        c = Config()
        _check("devirt_get_config", lib().devirt_get_config(self._h, ctypes.byref(c)))
        for k, v in kw.items():
            setattr(c, k, int(v))
        _check("devirt_set_config", lib().devirt_set_config(self._h, ctypes.byref(c)))

    def autotune(self, reqs, n, res, epoch_end=None, faults=None, n_faults=None, stream=None, reps=3):
        ep = None
        ne = 0
        if epoch_end is not None:
            ep = np.ascontiguousarray(np.asarray(epoch_end, dtype=np.uint64))
            ne = len(ep)
        best, ms = Config(), ctypes.c_double()
        _check("devirt_autotune", lib().devirt_autotune(
            self._h, _ptr(reqs), n, ep.ctypes.data if ep is not None else None, ne, _ptr(res), _ptr(faults),
            _ptr(n_faults), _stream(stream), reps, ctypes.byref(best), ctypes.byref(ms)))
        return best.as_dict(), ms.value

    def autotune_cached(self, cache_path: str, key: str, reqs, n, res, epoch_end=None, faults=None, n_faults=None,
                        stream=None, reps=3):
        """devirt_autotune_cached: returns (config, ms, hit)."""
        ep = None
        ne = 0
        if epoch_end is not None:
            ep = np.ascontiguousarray(np.asarray(epoch_end, dtype=np.uint64))
            ne = len(ep)
        best, ms, hit = Config(), ctypes.c_double(), ctypes.c_int()
        _check("devirt_autotune_cached", lib().devirt_autotune_cached(
            self._h, os.fsencode(cache_path), key.encode(), _ptr(reqs), n, ep.ctypes.data if ep is not None else None,
            ne, _ptr(res), _ptr(faults), _ptr(n_faults), _stream(stream), reps, ctypes.byref(best), ctypes.byref(ms),
            ctypes.byref(hit)))
        return best.as_dict(), ms.value, bool(hit.value)

    def set_profiling(self, on=True, counters: bool = True):
        """Timing events (and, unless counters=False, device counters); off when on is False."""
        flags = (PROF_TIMING | (PROF_COUNTERS if counters else 0)) if on else 0
        _check("devirt_set_profiling", lib().devirt_set_profiling(self._h, flags))

    def get_stats(self) -> dict:
        s = Stats()
        _check("devirt_get_stats", lib().devirt_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def reset_stats(self):
        _check("devirt_reset_stats", lib().devirt_reset_stats(self._h))

    def fifo_counts(self, asid: int):
        """(hits, misses) of the process's translation cache since the last flush."""
        h, m = u64(), u64()
        _check("devirt_fifo_counts", lib().devirt_fifo_counts(self._h, asid, ctypes.byref(h), ctypes.byref(m)))
        return int(h.value), int(m.value)

    def fifo_flush(self):
        _check("devirt_fifo_flush", lib().devirt_fifo_flush(self._h))

    # ---- serving
    def server_start(self, max_inflight=4096, pool_bytes=1 << 30, max_batch=0, streams=2, completion="poll",
                     device_times=False):
        """completion: "poll", "notify" or "blocking" (the DEVIRT_SERVE_* modes);
        device_times: completions carry their batch's device window."""
        cfg = ServerCfg(max_inflight, pool_bytes, max_batch, streams,
                        SERVE_MODES[completion] | (SERVE_DEVICE_TIMES if device_times else 0))
        h = vp()
        _check("devirt_server_start", lib().devirt_server_start(self._h, ctypes.byref(cfg), ctypes.byref(h)))
        return Server(h)


class Server:
    def __init__(self, h):
        self._h = h
        self._held = {}  # ticket -> result array of a map batch, written at completion

    def submit_map(self, asid: int, tag: int, maps: np.ndarray, pool_gpa) -> tuple:
        """Queue a map batch for guest thread (asid, tag); returns its ticket
        and the array that receives every map's result when it completes."""
        m = np.ascontiguousarray(maps, dtype=MAP_DTYPE)
        pool = np.ascontiguousarray(np.asarray(pool_gpa, dtype=np.uint64).reshape(-1))
        res = np.zeros(max(len(m), 1), RESULT_DTYPE)
        t = u64()
        _check("devirt_server_submit_map", lib().devirt_server_submit_map(
            self._h, asid, tag, m.ctypes.data if len(m) else None, len(m), pool.ctypes.data if len(pool) else None,
            len(pool), res.ctypes.data, ctypes.byref(t)))
        self._held[t.value] = res
        return t.value, res[:len(m)]

    def submit_ept_map(self, asid: int, tag: int, vm: int, maps: np.ndarray, pool) -> tuple:
        """Queue an EPT map batch of VM vm, in guest thread (asid, tag)'s order;
        returns its ticket and the array that receives every map's result."""
        m = np.ascontiguousarray(maps, dtype=EPT_MAP_DTYPE)
        pool = np.ascontiguousarray(np.asarray(pool, dtype=np.uint64).reshape(-1))
        res = np.zeros(max(len(m), 1), RESULT_DTYPE)
        t = u64()
        _check("devirt_server_submit_ept_map", lib().devirt_server_submit_ept_map(
            self._h, asid, tag, vm, m.ctypes.data if len(m) else None, len(m),
            pool.ctypes.data if len(pool) else None, len(pool), res.ctypes.data, ctypes.byref(t)))
        self._held[t.value] = res
        return t.value, res[:len(m)]

    def submit(self, reqs: np.ndarray) -> int:
        r = np.ascontiguousarray(reqs, dtype=REQUEST_DTYPE)
        n = u32()
        _check("devirt_server_submit", lib().devirt_server_submit(self._h, r.ctypes.data, len(r), ctypes.byref(n)))
        return n.value

    def poll(self, max_n: int = 4096, out: np.ndarray | None = None) -> np.ndarray:
        """Take up to max_n completions (into `out` when given, which is reused)."""
        if out is None or len(out) < max_n:
            out = np.empty(max_n, COMPLETION_DTYPE)
        n = u32()
        _check("devirt_server_poll", lib().devirt_server_poll(self._h, out.ctypes.data, max_n, ctypes.byref(n)))
        got = out[:n.value].copy()
        if self._held:  # a map batch's results are written by the time it completes
            for t in got["ticket"].tolist():
                self._held.pop(t, None)
        return got

    def drain(self):
        _check("devirt_server_drain", lib().devirt_server_drain(self._h))

    def stats(self) -> dict:
        st = ServerStats()
        _check("devirt_server_get_stats", lib().devirt_server_get_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def stop(self):
        if self._h:
            _check("devirt_server_stop", lib().devirt_server_stop(self._h))
            self._h = vp()
