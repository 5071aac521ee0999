"""The per-process FIFO translation cache of section 4.2 on the per-request
path: hits and misses equal the oracle's sequential FIFO exactly, on the
hand-derived sequence and on generated worlds and locality traces, and every
result, arena byte and host byte stays bit-exact."""
import numpy as np
import pytest

import pins
from gpu_util import log, new_ctx
from oracle import Oracle
from workload import device, gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _plain(ctx, reqs, res, stream):
    """Every request through the per-request path, in order, on one stream."""
    base = res.data_ptr()
    for i, r in enumerate(reqs):
        f = ctx.copy_to_guest if int(r["dir"]) == 1 else ctx.copy_from_guest
        f(int(r["asid"]), int(r["gva"]), int(r["host"]), int(r["len"]), base + 24 * i, stream)


def test_golden_fifo_sequence():
    """The hand-derived sequence: cumulative (hits, misses) after every copy."""
    import torch
    import paper_1304_3771_amd as dv
    H = pins.H
    world = [w for w in pins.golden_worlds() if "fifo" in w][0]
    o, arena, pool = pins.build_golden(world)
    ctx = new_ctx(fifo_entries=world["fifo"]["entries"])
    try:
        vm = ctx.vm_create(H(world["arena_bytes"]))
        ctx.vm_write(vm, 0, arena)
        for i, sl in enumerate(world["slots"]):
            ctx.memslot_set(vm, i, H(sl["gpa"]), H(sl["bytes"]), H(sl["arena_off"]))
        asid = ctx.process_create(vm, H(world["cr3"]), world["levels"])
        dpool = torch.from_numpy(pool.copy()).cuda()
        ctx.fifo_flush()
        res = torch.zeros(24, dtype=torch.uint8, device="cuda")
        o.fifo_reset(world["fifo"]["entries"])
        for k, st in enumerate(world["fifo"]["steps"]):
            f = ctx.copy_to_guest if st["dir"] == 1 else ctx.copy_from_guest
            f(asid, H(st["gva"]), dpool.data_ptr(), H(st["len"]), res)
            got = ctx.fifo_counts(asid)
            assert got == (st["hits"], st["misses"]), (k, got, st)
            req = np.zeros(1, dv.REQUEST_DTYPE)
            req[0] = (H(st["gva"]), 0, H(st["len"]), 0, st["dir"], (0, 0, 0), 0)
            er = o.copy(req[0])
            assert res.cpu().numpy().view(dv.RESULT_DTYPE)[0].tobytes() == er.tobytes(), k
        a = np.empty(H(world["arena_bytes"]), np.uint8)
        ctx.vm_read(vm, 0, a)
        assert np.array_equal(a, o.arenas[0])
        assert np.array_equal(dpool.cpu().numpy(), o.pool)
    finally:
        ctx.close()


@pytest.mark.parametrize("name,entries", [("mix2m", 10), ("prot", 10), ("multi_vm", 10), ("ept_faults", 10),
                                          ("pae_prot", 10), ("lvl5_1g", 10), ("mix2m", 9), ("multi_vm", 16),
                                          ("c1", 1)])
def test_fifo_counts_match_oracle(name, entries):
    """A locality trace (each process revisits a few buffers) and then the
    world's own requests, one at a time: per-process hits and misses, results,
    arenas and pool equal the oracle's."""
    import torch
    import paper_1304_3771_amd as dv
    w = gen.make_workload(pins.small_specs()[name])
    loc, loc_pool = gen.make_locality_trace(w, 4000, seed=5)
    reqs = np.concatenate([loc, w.requests_at(loc_pool)])
    pool_bytes = loc_pool + w.pool_bytes
    pool = gen.fill_bytes(np.empty(pool_bytes, np.uint8), w.seed, gen.POOL_KEY)
    o = Oracle.from_workload(w, pool=pool.copy())
    o.fifo_reset(entries)
    er, _ = o.batch(reqs)
    ctx = new_ctx(fifo_entries=entries)
    try:
        dw = device.load(ctx, w)
        dpool = torch.from_numpy(pool).cuda()
        hreq = reqs.copy()
        hreq["host"] += np.uint64(dpool.data_ptr())
        ctx.fifo_flush()
        res = torch.zeros(len(reqs) * 24, dtype=torch.uint8, device="cuda")
        _plain(ctx, hreq, res, torch.cuda.current_stream())
        ctx.sync()
        r = res.cpu().numpy().view(dv.RESULT_DTYPE)
        assert np.array_equal(r.view(np.uint8), er.view(np.uint8)), "results differ"
        for v, a in enumerate(device.read_arenas(ctx, dw)):
            assert np.array_equal(a, o.arenas[v]), f"vm {v} differs"
        assert np.array_equal(dpool.cpu().numpy(), o.pool)
        tot = [0, 0]
        for p in w.procs:
            got = ctx.fifo_counts(p.asid)
            exp = o.fifo_counts(p.asid)
            assert got == exp, (p.asid, got, exp)
            tot[0] += got[0]
            tot[1] += got[1]
        log(f"fifo {name}/{entries}: {tot[0]} hits, {tot[1]} misses, hit rate {tot[0] / max(1, sum(tot)):.3f}")
        assert tot[0] > 0
    finally:
        ctx.close()


def test_fifo_emptied_by_table_writes():
    """Writing guest memory (here: restoring the tables, which clears A/D
    bits) empties the caches: the same sequence run again misses as the first
    time and sets the A/D bits again, bit-exact."""
    import torch
    import paper_1304_3771_amd as dv
    w = gen.make_workload(pins.small_specs()["mix2m"])
    loc, loc_pool = gen.make_locality_trace(w, 1500, seed=6)
    pool = gen.fill_bytes(np.empty(loc_pool, np.uint8), w.seed, gen.POOL_KEY)
    ctx = new_ctx(fifo_entries=10)
    try:
        dw = device.load(ctx, w)
        dpool = torch.from_numpy(pool.copy()).cuda()
        hreq = loc.copy()
        hreq["host"] += np.uint64(dpool.data_ptr())
        res = torch.zeros(len(loc) * 24, dtype=torch.uint8, device="cuda")
        counts = []
        for rep in range(2):
            # back to the initial image: arenas and pool
            for v in w.vms:
                ctx.vm_write(v.vm, 0, w.arena_image(v.vm))
            dpool.copy_(torch.from_numpy(pool))
            h0 = ctx.fifo_counts(0)
            _plain(ctx, hreq, res, torch.cuda.current_stream())
            ctx.sync()
            h1 = ctx.fifo_counts(0)
            counts.append((h1[0] - h0[0], h1[1] - h0[1]))
            o = Oracle.from_workload(w, pool=pool.copy())
            o.fifo_reset(10)
            er, _ = o.batch(loc)
            assert np.array_equal(res.cpu().numpy().view(dv.RESULT_DTYPE).view(np.uint8), er.view(np.uint8))
            for v, a in enumerate(device.read_arenas(ctx, dw)):
                assert np.array_equal(a, o.arenas[v]), f"rep {rep}: vm {v} differs"
            assert (counts[-1][0], counts[-1][1]) == o.fifo_counts(0)
        assert counts[0] == counts[1]
    finally:
        ctx.close()
