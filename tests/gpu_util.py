"""Helpers for the GPU parity tests: run a workload through the C ABI and
through the oracle, and compare everything element by element."""
from __future__ import annotations

import sys

import numpy as np

from oracle import Oracle
from workload import device


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def new_ctx(**cfg):
    import paper_1304_3771_amd as dv
    ctx = dv.Context(0)
    if cfg:
        ctx.set_config(**cfg)
    return ctx


def gpu_batch(wl, cfg=None, epochs=True, t_done=False, ctx=None, dw=None, repeat=1):
    """Run the workload's requests as one submit_batch; return (res, faults, arenas, pool, extra)."""
    import torch
    import paper_1304_3771_amd as dv
    own = ctx is None
    if own:
        ctx = new_ctx(**(cfg or {}))
    try:
        if dw is None:
            dw = device.load(ctx, wl)
        n = dw.n
        res = torch.zeros(max(n, 1) * 24, dtype=torch.uint8, device="cuda")
        faults = torch.zeros(max(n, 1) * 24, dtype=torch.uint8, device="cuda")
        nf = torch.zeros(1, dtype=torch.int64, device="cuda")
        td = torch.zeros(max(n, 1), dtype=torch.int64, device="cuda") if t_done else None
        for _ in range(repeat):
            ctx.submit_batch(dw.reqs, n, res, wl.epoch_end if epochs else None, faults, nf, td)
        ctx.sync()
        torch.cuda.synchronize()
        r = res.cpu().numpy()[:n * 24].view(dv.RESULT_DTYPE)
        k = int(nf.item())
        f = faults.cpu().numpy()[:k * 24].view(dv.FAULT_DTYPE)
        arenas = device.read_arenas(ctx, dw)
        pool = dw.pool.cpu().numpy()
        extra = {"t_done": td.cpu().numpy()[:n] if t_done else None, "stats": ctx.get_stats()}
        return r, f, arenas, pool, extra
    finally:
        if own:
            ctx.close()


def oracle_batch(wl, reqs=None):
    o = Oracle.from_workload(wl)
    res, faults = o.batch(wl.requests if reqs is None else reqs)
    return res, faults, o.arenas, o.pool


def compare(tag, got, exp):
    """Element-by-element comparison of (res, faults, arenas, pool)."""
    r, f, a, p = got[:4]
    er, ef, ea, ep = exp[:4]
    errs = []
    for fld in ("bytes_done", "fault_gva", "code", "level"):
        if not np.array_equal(r[fld], er[fld]):
            i = int(np.nonzero(r[fld] != er[fld])[0][0])
            errs.append(f"{tag}: result.{fld} differs at request {i}: gpu {r[i]} oracle {er[i]}")
            break
    if len(f) != len(ef):
        errs.append(f"{tag}: {len(f)} faults on the GPU, {len(ef)} in the oracle")
    else:
        for fld in ("req_index", "fault_gva", "code", "level"):
            if not np.array_equal(f[fld], ef[fld]):
                errs.append(f"{tag}: fault list field {fld} differs")
                break
    for v, (x, y) in enumerate(zip(a, ea)):
        if not np.array_equal(x, y):
            bad = np.nonzero(x != y)[0]
            errs.append(f"{tag}: vm {v} arena differs in {len(bad)} bytes, first at {hex(int(bad[0]))}")
    if not np.array_equal(p, ep):
        bad = np.nonzero(p != ep)[0]
        errs.append(f"{tag}: pool differs in {len(bad)} bytes, first at {int(bad[0])}")
    return errs
