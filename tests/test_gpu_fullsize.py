"""Full-size parity: the one-guest 4 GiB workload with 1e6 requests (64 B - 64 KiB,
70/30 4 KiB/2 MiB pages, 16 memslots, 5% not present), run as the benchmark
runs it (HIP graph, all epochs), once in the default launch configuration and
once in the configuration the autotuner picks -- the one the benchmark
times -- compared with the oracle on every result, every fault record, every
arena byte (A/D bits included) and every host-buffer byte."""
import numpy as np
import pytest

from gpu_util import log, new_ctx
from oracle import Oracle
from workload import device, gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2_expected():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    log("full C2: generating and running the oracle")
    wl = gen.make_workload(gen.spec("C2"))
    o = Oracle.from_workload(wl)
    er, ef = o.batch(wl.requests)
    return wl, o, er, ef


def _restore(ctx, wl, dw):
    """Write every arena byte and every host-buffer byte back to the initial image."""
    import torch
    for v in wl.vms:
        img = wl.arena_image(v.vm)
        chunk = 1 << 30
        for off in range(0, v.arena_bytes, chunk):
            m = min(chunk, v.arena_bytes - off)
            ctx.vm_write(v.vm, off, img[off:off + m], m)
        del img
    dw.pool.copy_(torch.from_numpy(wl.pool_image()))
    torch.cuda.synchronize()


@pytest.mark.parametrize("launch", ["default", "autotuned"])
def test_full_c2_bit_exact(c2_expected, launch):
    import torch
    import paper_1304_3771_amd as dv
    wl, o, er, ef = c2_expected
    n = wl.n_requests
    ctx = new_ctx()
    try:
        dw = device.load(ctx, wl)
        res = torch.zeros(n * 24, dtype=torch.uint8, device="cuda")
        faults = torch.zeros(n * 24, dtype=torch.uint8, device="cuda")
        nf = torch.zeros(1, dtype=torch.int64, device="cuda")
        if launch == "autotuned":
            # the benchmark's own call; tuning runs the batch several times
            best, ms = ctx.autotune(dw.reqs, n, res, wl.epoch_end, faults, nf, reps=3)
            log(f"full C2: autotuned {best} ({ms:.3f} ms); restoring memory")
            _restore(ctx, wl, dw)
            res.zero_()
            faults.zero_()
            nf.zero_()
        log(f"full C2 ({launch}): running the batch with {ctx.get_config()}")
        ctx.submit_batch(dw.reqs, n, res, wl.epoch_end, faults, nf)
        ctx.sync()
        r = res.cpu().numpy().view(dv.RESULT_DTYPE)
        k = int(nf.item())
        f = faults.cpu().numpy()[:24 * k].view(dv.FAULT_DTYPE)
        assert np.array_equal(r.view(np.uint8), er.view(np.uint8)), "results differ"
        assert np.array_equal(f.view(np.uint8), ef.view(np.uint8)), "fault lists differ"
        arena = device.read_arenas(ctx, dw)[0]
        bad = np.count_nonzero(arena != o.arenas[0])
        assert bad == 0, f"{bad} arena bytes differ"
        del arena
        chunk = 1 << 30
        for off in range(0, wl.pool_bytes, chunk):
            m = min(chunk, wl.pool_bytes - off)
            got = dw.pool[off:off + m].cpu().numpy()
            assert np.array_equal(got, o.pool[off:off + m]), f"pool differs in [{off}, {off + m})"
        log(f"full C2 ({launch}): bit-exact ({n} requests, {k} faults, {int(r['bytes_done'].sum())} bytes)")
    finally:
        ctx.close()


def _pt_frames(ctx, wl):
    """Read every page-table frame of every VM back from the GPU arenas."""
    out = {}
    for v in wl.vms:
        hpa = gen.gpa_to_arena(v.slots, v.pt_gfn << np.uint64(12))
        buf = np.empty((len(hpa), 4096), np.uint8)
        order = np.argsort(hpa)
        i = 0
        while i < len(order):
            j = i + 1
            while j < len(order) and hpa[order[j]] == hpa[order[j - 1]] + 4096:
                j += 1
            tmp = np.empty((j - i) * 4096, np.uint8)
            ctx.vm_read(v.vm, int(hpa[order[i]]), tmp, tmp.size)
            buf[order[i:j]] = tmp.reshape(-1, 4096)
            i = j
        out[v.vm] = buf.view(np.uint64)
    return out


def _restore_tables(ctx, wl):
    """Write every page-table frame back (clears the A/D bits earlier runs set)."""
    for v in wl.vms:
        hpa = gen.gpa_to_arena(v.slots, v.pt_gfn << np.uint64(12))
        for i in np.argsort(hpa):
            blk = np.ascontiguousarray(v.pt_data[i]).view(np.uint8)
            ctx.vm_write(v.vm, int(hpa[i]), blk, blk.size)


def _tables_only_oracle(wl):
    """Oracle state with page-table frames only (enough for results: the data
    bytes never influence a translation).  np.zeros pages stay unmaterialised."""
    arenas = []
    for v in wl.vms:
        a = np.zeros(v.arena_bytes, np.uint8)
        wl.overlay_tables(v.vm, a)
        if v.ept_root is not None:
            a.reshape(-1, 4096)[(v.ept_off >> np.uint64(12)).astype(np.int64)] = \
                v.ept_data.view(np.uint8).reshape(-1, 4096)
        arenas.append(a)
    return Oracle(arenas, [v.slots for v in wl.vms], [(p.vm, p.cr3, p.levels) for p in wl.procs],
                  np.zeros(4096, np.uint8), ept=[v.ept_root for v in wl.vms])


_FULL = {"C3": gen.spec("C3"), "C5": gen.spec("C5"),
         # C2's shape with its guest-physical space behind a 4-level EPT (as the C2-EPT benchmark)
         "C2-EPT": gen.spec("C2", ept=True, seed=1007)}


@pytest.mark.parametrize("name", ["C3", "C5", "C2-EPT"])
def test_full_size_results_and_ad(name):
    """16 VMs x 4 processes x 2 GiB, 4e6 requests 16 B-4 MiB (C3), 64 VMs x 2 GiB with
    5-level paging and 1 GiB pages, 1e7 requests (C5), or C2 behind an EPT, run as the
    benchmark runs them:
    autotuned launch configuration, HIP graph, all epochs.
    Checked: every 29th request's result against the oracle (exact), the fault list is
    the ascending list of faulting requests with their records, A/D bits of every table
    entry (set exactly where the sampled copies demand, never outside any request's
    range, no other bit changed)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1304_3771_amd as dv
    from pins import _leaf_lookup, find_leaf
    log(f"full {name}: generating")
    wl = gen.make_workload(_FULL[name])
    n = wl.n_requests
    ctx = new_ctx()
    try:
        dw = device.load(ctx, wl)
        log(f"full {name}: uploaded, {n} requests in {len(wl.epoch_end)} epochs")
        res = torch.zeros(n * 24, dtype=torch.uint8, device="cuda")
        faults = torch.zeros(n * 24, dtype=torch.uint8, device="cuda")
        nf = torch.zeros(1, dtype=torch.int64, device="cuda")
        # the benchmark's own tuning call; it runs the batch several times, so the
        # tables (the only state results depend on) are written back afterwards
        best, ms = ctx.autotune(dw.reqs, n, res, wl.epoch_end, faults, nf, reps=1)
        log(f"full {name}: autotuned {best} ({ms:.1f} ms); restoring the tables")
        _restore_tables(ctx, wl)
        res.zero_()
        faults.zero_()
        nf.zero_()
        torch.cuda.synchronize()
        ctx.submit_batch(dw.reqs, n, res, wl.epoch_end, faults, nf)
        ctx.sync()
        r = res.cpu().numpy().view(dv.RESULT_DTYPE)
        k = int(nf.item())
        f = faults.cpu().numpy()[:24 * k].view(dv.FAULT_DTYPE)
        tables = _pt_frames(ctx, wl)
    finally:
        ctx.close()
    # fault list: exactly the faulting requests, ascending, with their records
    fidx = np.nonzero(r["code"] != 0)[0]
    assert np.array_equal(f["req_index"], fidx.astype(np.uint64))
    for fld in ("fault_gva", "code", "level"):
        assert np.array_equal(f[fld], r[fld][fidx])
    # sampled results, exact
    log(f"full {name}: oracle results for a 1/29 sample")
    o = _tables_only_oracle(wl)
    sel = np.arange(0, n, 29)
    er, _ = o.batch_results(wl.requests[sel])
    assert np.array_equal(r[sel].view(np.uint8).reshape(-1, 24), er.view(np.uint8).reshape(-1, 24))
    # A/D: only bits 5 and 6 may change, and only ever from 0 to 1
    for v in wl.vms:
        init = v.pt_data
        got = tables[v.vm]
        assert np.all((got & ~np.uint64(0x60)) == (init & ~np.uint64(0x60))), f"vm {v.vm}: non-A/D bits changed"
        assert np.all((got & init) == init), f"vm {v.vm}: an A/D bit was cleared"
    # leaves no request range touches stay exactly as written
    A, D = np.uint64(0x20), np.uint64(0x40)
    pos = {v.vm: (np.sort(v.pt_gfn), np.argsort(v.pt_gfn)) for v in wl.vms}
    for p in wl.procs:
        m = wl.requests["asid"] == p.asid
        lo = wl.requests["gva"][m]
        hi = lo + wl.requests["len"][m].astype(np.uint64)
        order = np.argsort(lo)
        lo, hi = lo[order], np.maximum.accumulate(hi[order])
        size = np.uint64(1) << (np.uint64(12) + np.uint64(9) * (p.leaf_level.astype(np.uint64) - np.uint64(1)))
        # any request range [lo, hi) intersecting [leaf, leaf + size)?
        j = np.searchsorted(lo, p.leaf_va + size, side="left") - 1
        touched = (j >= 0) & (hi[np.maximum(j, 0)] > p.leaf_va)
        gfns, ordr = pos[p.vm]
        row = ordr[np.searchsorted(gfns, p.leaf_table_gfn)]
        vals = tables[p.vm][row, p.leaf_index.astype(np.int64)]
        untouched = ~touched
        assert np.all(vals[untouched] == p.leaf_entry[untouched]), f"asid {p.asid}: an untouched leaf changed"
    # every copied page of the sampled requests: A on its leaf and D when written
    tabs = {}
    for i, rr in zip(sel, er):
        done = int(rr["bytes_done"])
        if done == 0:
            continue
        q = wl.requests[i]
        p = wl.procs[int(q["asid"])]
        if p.asid not in tabs:
            tabs[p.asid] = _leaf_lookup(p)
        g = int(q["gva"])
        pages = np.arange(g >> 12, ((g + done - 1) >> 12) + 1, dtype=np.uint64) << np.uint64(12)
        li = find_leaf(p, tabs[p.asid], pages)
        gfns, ordr = pos[p.vm]
        row = ordr[np.searchsorted(gfns, p.leaf_table_gfn[li])]
        vals = tables[p.vm][row, p.leaf_index[li].astype(np.int64)]
        assert np.all(vals & A), f"request {i}: a copied page's leaf lacks A"
        if int(q["dir"]) == 1:
            assert np.all(vals & D), f"request {i}: a written page's leaf lacks D"
    log(f"full {name}: ok ({k} faults, {int(r['bytes_done'].sum())} bytes copied)")
