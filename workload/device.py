"""Load a generated workload into a devirt context on the GPU.

Harness code: it creates the VMs, memslots and processes through the C ABI,
uploads each arena image (fill bytes + page-table frames) and places the
host-buffer pool and the request descriptors in HBM as torch tensors.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .gen import REQ_DTYPE, Workload


@dataclass
class DeviceWorkload:
    wl: Workload
    pool: object          # torch uint8 tensor on the device
    reqs: object          # torch uint8 tensor, n x 32 bytes
    reqs_host: np.ndarray  # the descriptors as uploaded (host = device pointers)
    vms: list

    @property
    def n(self) -> int:
        return len(self.reqs_host)


def load(ctx, wl: Workload, device: str = "cuda:0", arena_chunk: int = 1 << 30) -> DeviceWorkload:
    import torch

    vms = []
    buf = None
    for v in wl.vms:
        vm = ctx.vm_create(v.arena_bytes)
        if vm != v.vm:
            raise RuntimeError(f"VM ids out of step: got {vm}, generator expects {v.vm}")
        for i, s in enumerate(v.slots):
            ctx.memslot_set(vm, i, int(s["gpa"]), int(s["bytes"]), int(s["arena_off"]))
        if v.ept_root is not None:
            ctx.vm_set_ept(vm, v.ept_root)
        if buf is None or buf.size < v.arena_bytes:
            buf = np.empty(v.arena_bytes, np.uint8)
        img = buf[:v.arena_bytes]
        wl.arena_image(v.vm, out=img)
        for off in range(0, v.arena_bytes, arena_chunk):
            n = min(arena_chunk, v.arena_bytes - off)
            ctx.vm_write(vm, off, img[off:off + n], n)
        vms.append(vm)
    del buf
    for p in wl.procs:
        a = ctx.process_create(p.vm, p.cr3, p.levels)
        if a != p.asid:
            raise RuntimeError(f"asids out of step: got {a}, generator expects {p.asid}")
    pool = torch.from_numpy(wl.pool_image()).to(device) if wl.pool_bytes else \
        torch.zeros(4096, dtype=torch.uint8, device=device)
    reqs_host = wl.requests_at(pool.data_ptr())
    reqs = torch.from_numpy(reqs_host.view(np.uint8).reshape(-1)).to(device) if len(reqs_host) else \
        torch.zeros(32, dtype=torch.uint8, device=device)
    torch.cuda.synchronize()
    return DeviceWorkload(wl, pool, reqs, reqs_host, vms)


def read_arenas(ctx, dw: DeviceWorkload) -> list:
    out = []
    for v in dw.wl.vms:
        a = np.empty(v.arena_bytes, np.uint8)
        ctx.vm_read(v.vm, 0, a, v.arena_bytes)
        out.append(a)
    return out


def upload_requests(reqs: np.ndarray, device: str = "cuda:0"):
    import torch
    r = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
    return torch.from_numpy(r.view(np.uint8).reshape(-1).copy()).to(device)
