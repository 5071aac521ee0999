"""devirt_map_pages on the GPU vs the oracle, through the C ABI.

Bar: bit-exact: per-map results, the number of pool frames used and every
arena byte (new tables, links, leaves, and nothing else).
"""
import numpy as np
import pytest

import pins
from gpu_util import compare, log, new_ctx
from oracle import Oracle
from workload import device, gen

pytestmark = pytest.mark.gpu

SPECS = pins.small_specs()
_WL = {}


def wl(name):
    if name not in _WL:
        _WL[name] = gen.make_workload(SPECS[name])
    return _WL[name]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1304_3771_amd as dv
    dv.lib()


def _gpu_map(ctx, asid, m, pool):
    """One devirt_map_pages call; returns (results, frames used)."""
    import torch
    import paper_1304_3771_amd as dv
    n = len(m)
    dm = torch.from_numpy(np.ascontiguousarray(m).view(np.uint8).reshape(-1).copy()).cuda() if n else \
        torch.zeros(24, dtype=torch.uint8, device="cuda")
    res = torch.zeros(max(n, 1) * 24, dtype=torch.uint8, device="cuda")
    used = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    ctx.map_pages(asid, dm, n, pool, res, used)
    torch.cuda.synchronize()
    return res.cpu().numpy()[:n * 24].view(dv.RESULT_DTYPE), int(used.item())


def _same(tag, r, used, er, eused, arenas, earenas):
    errs = []
    for fld in ("bytes_done", "fault_gva", "code", "level"):
        if not np.array_equal(r[fld], er[fld]):
            i = int(np.nonzero(r[fld] != er[fld])[0][0])
            errs.append(f"{tag}: result.{fld} differs at map {i}: gpu {r[i]} oracle {er[i]}")
    if used != eused:
        errs.append(f"{tag}: {used} frames used on the GPU, {eused} in the oracle")
    for v, (a, b) in enumerate(zip(arenas, earenas)):
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            errs.append(f"{tag}: vm {v}: {len(bad)} arena bytes differ, first at {hex(int(bad[0]))}")
    assert not errs, "\n".join(errs)


def _golden_map_worlds():
    return [w for w in pins.golden_worlds() if "maps" in w]


@pytest.mark.parametrize("widx", range(len(_golden_map_worlds())))
def test_golden_maps(widx):
    """The hand-derived map batches (their expectations pin the oracle)."""
    import torch
    from oracle.oracle import MAP_DTYPE
    w = _golden_map_worlds()[widx]
    log(f"golden maps {w['name']}")
    H = pins.H
    o, arena, _ = pins.build_golden(w)
    ctx = new_ctx()
    try:
        vm = ctx.vm_create(H(w["arena_bytes"]))
        ctx.vm_write(vm, 0, arena)
        for i, s in enumerate(w["slots"]):
            ctx.memslot_set(vm, i, H(s["gpa"]), H(s["bytes"]), H(s["arena_off"]))
        if "ept_root" in w:
            ctx.vm_set_ept(vm, H(w["ept_root"]))
        assert ctx.process_create(vm, H(w["cr3"]), w["levels"]) == 0
        gm = w["maps"]
        m = np.zeros(len(gm["batch"]), MAP_DTYPE)
        for i, b in enumerate(gm["batch"]):
            m[i] = (H(b["gva"]), H(b["gpa"]), b["flags"], 0)
        pool = [H(x) for x in gm["pool"]]
        r, used = _gpu_map(ctx, 0, m, pool)
        er, eused = o.map_pages(0, m, pool)
        a = np.empty(H(w["arena_bytes"]), np.uint8)
        ctx.vm_read(vm, 0, a)
        _same(w["name"], r, used, er, eused, [a], [arena])
        assert used == gm["used"]
        torch.cuda.synchronize()
    finally:
        ctx.close()


@pytest.mark.parametrize("name", ["c1", "mix2m", "lvl5", "lvl5_1g", "pae", "pae_prot", "multi_vm", "ept",
                                  "ept_faults", "ept_pae"])
def test_map_matches_oracle(name):
    """A mixed batch (remaps, new regions, pages inside large leaves, out of
    range, duplicates): a too-small pool first (nothing written), then enough,
    then the same batch again (every table now exists), then the workload's
    requests through the new tables."""
    w = wl(name)
    log(f"map {name}")
    rng = np.random.default_rng(11)
    m = pins.map_batch(w, rng)
    vm = w.procs[0].vm
    pool = pins.usable_frames(w, vm, pins.free_frames(w, vm, 4 * len(m), rng))
    o = Oracle.from_workload(w)
    ctx = new_ctx()
    try:
        dw = device.load(ctx, w)
        # how many tables the batch needs, from a copy of the oracle
        _, need = Oracle.from_workload(w).map_pages(0, m, pool)
        assert need > 0
        r, used = _gpu_map(ctx, 0, m, pool[:need - 1])
        er, eused = o.map_pages(0, m, pool[:need - 1])
        _same(f"{name} short pool", r, used, er, eused, device.read_arenas(ctx, dw), o.arenas)
        assert used == 0 and np.any(r["code"] == pins.CODES["NO_POOL"])
        r, used = _gpu_map(ctx, 0, m, pool)
        er, eused = o.map_pages(0, m, pool)
        _same(f"{name} map", r, used, er, eused, device.read_arenas(ctx, dw), o.arenas)
        assert used == need
        r, used = _gpu_map(ctx, 0, m[::-1].copy(), pool[need:])
        er, eused = o.map_pages(0, m[::-1].copy(), pool[need:])
        _same(f"{name} again", r, used, er, eused, device.read_arenas(ctx, dw), o.arenas)
        assert used == 0
        # remapped pages may now alias other requests' bytes, so the
        # workload's epochs no longer separate conflicting requests: one
        # request per epoch keeps the batch's precondition
        import torch
        import paper_1304_3771_amd as dv
        n = dw.n
        res = torch.zeros(n * 24, dtype=torch.uint8, device="cuda")
        faults = torch.zeros(n * 24, dtype=torch.uint8, device="cuda")
        nf = torch.zeros(1, dtype=torch.int64, device="cuda")
        ctx.submit_batch(dw.reqs, n, res, np.arange(1, n + 1, dtype=np.uint64), faults, nf)
        ctx.sync()
        k = int(nf.item())
        got = (res.cpu().numpy()[:n * 24].view(dv.RESULT_DTYPE), faults.cpu().numpy()[:k * 24].view(dv.FAULT_DTYPE),
               device.read_arenas(ctx, dw), dw.pool.cpu().numpy())
        eres, efaults = o.batch(w.requests)
        assert compare(f"{name} batch after map", got, (eres, efaults, o.arenas, o.pool)) == []
    finally:
        ctx.close()


@pytest.mark.parametrize("name,n_pool", [("mix2m", 4096), ("lvl5_1g", 40000)])
def test_map_large_batch(name, n_pool):
    """2^17 maps in one call, half into a 4 GiB region the tables do not cover
    yet, half onto mapped pages.  The small pool has the new tables ordered in
    LDS tiles, the large one (over 2^14 frames) by LDS tiles and merge rounds."""
    w = wl(name)
    log(f"map large {name} pool {n_pool}")
    rng = np.random.default_rng(5)
    from oracle.oracle import MAP_DTYPE
    p = w.procs[0]
    n = 1 << 17
    m = np.zeros(n, MAP_DTYPE)
    base = np.uint64(0x7000_0000_0000)
    m["gva"][: n // 2] = base + (rng.integers(0, 1 << 20, n // 2).astype(np.uint64) << np.uint64(12))
    m["gva"][n // 2:] = p.leaf_va[rng.integers(0, len(p.leaf_va), n // 2)] & ~np.uint64(0xFFF)
    m["gpa"] = rng.integers(0, w.vms[p.vm].mem_bytes >> 12, n).astype(np.uint64) << np.uint64(12)
    m["flags"] = rng.integers(0, 2, n)
    pool = pins.free_frames(w, p.vm, n_pool, rng)
    o = Oracle.from_workload(w)
    ctx = new_ctx()
    try:
        dw = device.load(ctx, w)
        r, used = _gpu_map(ctx, 0, m, pool)
        er, eused = o.map_pages(0, m, pool)
        _same("large", r, used, er, eused, device.read_arenas(ctx, dw), o.arenas)
        assert used > 0
    finally:
        ctx.close()


def test_map_edge_cases():
    import paper_1304_3771_amd as dv
    from oracle.oracle import MAP_DTYPE
    w = wl("c1")
    log("map edges")
    rng = np.random.default_rng(2)
    p = w.procs[0]
    ctx = new_ctx()
    try:
        dw = device.load(ctx, w)
        a0 = device.read_arenas(ctx, dw)
        # no maps
        r, used = _gpu_map(ctx, 0, np.zeros(0, MAP_DTYPE), [])
        assert used == 0
        m = pins.map_batch(w, rng, n=60)
        # an asid with no process: every map INVALID, nothing written
        r, used = _gpu_map(ctx, len(w.procs), m, pins.free_frames(w, p.vm, 8, rng))
        assert used == 0 and np.all(r["code"] == pins.CODES["INVALID"])
        assert np.array_equal(r["fault_gva"], m["gva"])
        # no pool at all
        o = Oracle.from_workload(w)
        r, used = _gpu_map(ctx, 0, m, [])
        er, eused = o.map_pages(0, m, [])
        _same("no pool", r, used, er, eused, device.read_arenas(ctx, dw), o.arenas)
        assert all(np.array_equal(a, b) for a, b in zip(a0, device.read_arenas(ctx, dw)))
        # rejected pools: unaligned, outside every memslot, repeated
        import torch
        dm = torch.from_numpy(m.view(np.uint8).copy()).cuda()
        res = torch.zeros(len(m) * 24, dtype=torch.uint8, device="cuda")
        nu = torch.zeros(1, dtype=torch.int64, device="cuda")
        good = pins.free_frames(w, p.vm, 2, rng)
        for bad in ([int(good[0]) + 8], [1 << 51], [int(good[0]), int(good[1]), int(good[0])]):
            with pytest.raises(dv.DevirtError) as ei:
                ctx.map_pages(0, dm, len(m), bad, res, nu)
            assert ei.value.rc == -22
        with pytest.raises(dv.DevirtError) as ei:
            ctx.map_pages(0, dm, (1 << 19) + 1, [], res, nu)
        assert ei.value.rc == -22
        torch.cuda.synchronize()
        assert all(np.array_equal(a, b) for a, b in zip(a0, device.read_arenas(ctx, dw)))
    finally:
        ctx.close()


def test_map_ept_bad_pool_frame():
    """EPT VM: a pool frame the batch takes that the EPT does not map readable
    and writable fails the batch (NO_POOL, nothing written); past the frames
    the batch takes it changes nothing.  Compared with the oracle."""
    from workload.gen import EPT_LEAF_NP, EPT_LEAF_OK, EPT_LEAF_RO
    w = wl("ept_faults")
    log("map: EPT VM, bad pool frames")
    rng = np.random.default_rng(8)
    p = w.procs[0]
    lf = w.vms[p.vm].ept_leaf
    m = pins.map_batch(w, rng)
    cand = pins.free_frames(w, p.vm, 4000, rng)
    kind = lf["kind"][np.searchsorted(lf["gpa"], cand, side="right") - 1]
    good = cand[kind == EPT_LEAF_OK]
    _, need = Oracle.from_workload(w).map_pages(0, m, good)
    assert need >= 2
    pools = [np.concatenate([good[:need // 2], cand[kind == k][:1], good[need // 2:]]) for k in (EPT_LEAF_NP, EPT_LEAF_RO)]
    pools.append(np.concatenate([good[:need], cand[kind == EPT_LEAF_NP][:1]]))
    o = Oracle.from_workload(w)
    ctx = new_ctx()
    try:
        dw = device.load(ctx, w)
        for k, pool in enumerate(pools):
            r, used = _gpu_map(ctx, 0, m, pool)
            er, eused = o.map_pages(0, m, pool)
            _same(f"bad pool {k}", r, used, er, eused, device.read_arenas(ctx, dw), o.arenas)
            assert (used == 0) == (k < 2)
    finally:
        ctx.close()


def test_map_full_size_c2():
    """At the benchmark's size: 2^19 maps per call on C2's tables (4 GiB guest),
    a fresh batch then a remap batch as the benchmark makes them; results,
    frames used and every arena byte against the oracle."""
    import sys
    import torch
    import os
    import paper_1304_3771_amd as dv
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    log("map full size: generating C2")
    w = gen.make_workload(gen.spec("C2"), requests=False)
    p = w.procs[0]
    n = 1 << 19
    mem = w.vms[p.vm].mem_bytes >> 12
    free = bench.free_guest_frames(w, p.vm)
    rng = np.random.default_rng(21)
    batches = [bench.map_fresh_batch(rng, n, 1 << 47, mem, dv.MAP_DTYPE, dv.MAP_WRITE),
               bench.map_remap_batch(rng, n, p, mem, dv.MAP_DTYPE)]
    o = Oracle.from_workload(w)
    ctx = new_ctx()
    try:
        dw = device.load(ctx, w)
        log("map full size: uploaded")
        nxt = 0
        for k, m in enumerate(batches):
            pool = free[nxt:nxt + 4096]
            r, used = _gpu_map(ctx, 0, m, pool)
            er, eused = o.map_pages(0, m, pool)
            assert np.array_equal(r.view(np.uint8), er.view(np.uint8)), f"batch {k}: results differ"
            assert used == eused and (used > 0) == (k == 0), (k, used, eused)
            nxt += used
        torch.cuda.synchronize()
        a = device.read_arenas(ctx, dw)[0]
        bad = np.count_nonzero(a != o.arenas[0])
        assert bad == 0, f"{bad} arena bytes differ"
        log(f"map full size: bit-exact, {nxt} new tables")
    finally:
        ctx.close()


def test_map_scattered_many_tables():
    """2^16 maps at random pages across 64 TiB of the address space: nearly
    every map needs its own page table and page directory, so over 10^5 new
    tables are ordered by LDS tiles and eight merge rounds.  With the pool
    one short of that, nothing is written; with enough, results, frames used
    and every arena byte equal the oracle."""
    import torch
    import os
    import sys
    import paper_1304_3771_amd as dv
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    log("map scattered: generating C2")
    w = gen.make_workload(gen.spec("C2"), requests=False)
    p = w.procs[0]
    n = 1 << 16
    rng = np.random.default_rng(23)
    m = np.zeros(n, dv.MAP_DTYPE)
    m["gva"] = (np.uint64(1 << 40) + (rng.integers(0, (1 << 46) >> 12, n).astype(np.uint64) << np.uint64(12)))
    m["gpa"] = rng.integers(0, w.vms[p.vm].mem_bytes >> 12, n).astype(np.uint64) << np.uint64(12)
    m["flags"] = rng.integers(0, 2, n)
    free = bench.free_guest_frames(w, p.vm)
    _, need = Oracle.from_workload(w).map_pages(0, m, free[:4 * n])
    assert need > 100_000 and len(free) >= 4 * n
    o = Oracle.from_workload(w)
    ctx = new_ctx()
    try:
        dw = device.load(ctx, w)
        for pool in (free[:need - 1], free[:150_000]):
            r, used = _gpu_map(ctx, 0, m, pool)
            er, eused = o.map_pages(0, m, pool)
            assert np.array_equal(r.view(np.uint8), er.view(np.uint8)), f"pool {len(pool)}: results differ"
            assert used == eused == (need if len(pool) >= need else 0), (used, eused, need)
        torch.cuda.synchronize()
        a = device.read_arenas(ctx, dw)[0]
        bad = np.count_nonzero(a != o.arenas[0])
        assert bad == 0, f"{bad} arena bytes differ"
        log(f"map scattered: bit-exact, {need} new tables")
    finally:
        ctx.close()


# ------------------------------------------------------------- EPT maps --
def _gpu_ept_map(ctx, vm, m, pool):
    """One devirt_ept_map_pages call; returns (results, pool pages used)."""
    import torch
    import paper_1304_3771_amd as dv
    n = len(m)
    dm = torch.from_numpy(np.ascontiguousarray(m).view(np.uint8).reshape(-1).copy()).cuda() if n else \
        torch.zeros(24, dtype=torch.uint8, device="cuda")
    res = torch.zeros(max(n, 1) * 24, dtype=torch.uint8, device="cuda")
    used = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    ctx.ept_map_pages(vm, dm, n, pool, res, used)
    torch.cuda.synchronize()
    return res.cpu().numpy()[:n * 24].view(dv.RESULT_DTYPE), int(used.item())


def test_golden_ept_maps():
    """The hand-derived EPT map batch (its expectations pin the oracle), then
    the same batch with the pool one page short (nothing written)."""
    from oracle.oracle import EPT_MAP_DTYPE
    H = pins.H
    w = [x for x in pins.golden_worlds() if "ept_maps" in x][0]
    gm = w["ept_maps"]
    m = np.zeros(len(gm["batch"]), EPT_MAP_DTYPE)
    for i, b in enumerate(gm["batch"]):
        m[i] = (H(b["gpa"]), H(b["hpa"]), b["flags"], 0)
    for pool_key in ("pool", "short_pool"):
        log(f"golden EPT maps, {pool_key}")
        o, arena, _ = pins.build_golden(w)
        ctx = new_ctx()
        try:
            vm = ctx.vm_create(H(w["arena_bytes"]))
            ctx.vm_write(vm, 0, arena)
            ctx.vm_set_ept(vm, H(w["ept_root"]))
            pool = [H(x) for x in gm[pool_key]]
            r, used = _gpu_ept_map(ctx, vm, m, pool)
            er, eused = o.ept_map_pages(0, m, pool)
            a = np.empty(H(w["arena_bytes"]), np.uint8)
            ctx.vm_read(vm, 0, a)
            _same(f"golden EPT maps {pool_key}", r, used, er, eused, [a], [arena])
            assert used == (gm["used"] if pool_key == "pool" else 0)
        finally:
            ctx.close()


@pytest.mark.parametrize("name", ["ept", "ept_faults", "ept_lvl5", "ept_pae", "ept_1g"])
def test_ept_map_matches_oracle(name):
    """A mixed EPT map batch (pages inside guest memory, new regions far above
    it, pages inside 2 MiB / 1 GiB EPT leaves, repeats, invalid maps): a pool
    one page short (nothing written), then enough, then the same batch again
    (every table now exists), then the workload's requests through the
    changed EPT; results, pages used and every arena byte, and the batch's
    results, fault list, arenas and pool."""
    from gpu_util import gpu_batch
    w = wl(name)
    log(f"EPT map {name}")
    rng = np.random.default_rng(7)
    vm = 0
    m, pool = pins.ept_map_batch(w, vm, 400, rng)
    o = Oracle.from_workload(w)
    ctx = new_ctx()
    try:
        dw = device.load(ctx, w)
        _, need = Oracle.from_workload(w).ept_map_pages(vm, m, pool)
        assert need > 0
        for k, p in enumerate((pool[:need - 1], pool, pool)):
            r, used = _gpu_ept_map(ctx, vm, m, p)
            er, eused = o.ept_map_pages(vm, m, p)
            _same(f"{name} EPT map call {k}", r, used, er, eused, device.read_arenas(ctx, dw), o.arenas)
            log(f"call {k}: {used} pages used, {int(np.count_nonzero(r['code'] == 0))} maps ok")
        got = gpu_batch(w, ctx=ctx, dw=dw)
        er, ef = o.batch(w.requests)
        assert compare(f"{name} requests after EPT maps", got, (er, ef, o.arenas, o.pool)) == []
    finally:
        ctx.close()


def test_ept_map_edge_cases():
    """Refused with nothing done: a VM without an EPT, an unknown VM, pool
    pages unaligned, outside the arena or repeated, too many maps; an empty
    batch writes nothing and uses no page."""
    import paper_1304_3771_amd as dv
    from oracle.oracle import EPT_MAP_DTYPE
    w = wl("ept")
    ctx = new_ctx()
    try:
        dw = device.load(ctx, w)
        before = device.read_arenas(ctx, dw)
        arena = w.vms[0].arena_bytes
        m = np.zeros(1, EPT_MAP_DTYPE)
        m[0] = (0x1000, 0x1000, 3, 0)
        for vm, pool in ((5, [0x10000]), (0, [0x10001]), (0, [arena]), (0, [0x10000, 0x10000])):
            with pytest.raises(dv.DevirtError):
                _gpu_ept_map(ctx, vm, m, pool)
        with pytest.raises(dv.DevirtError):
            ctx.ept_map_pages(0, 0, (1 << 19) + 1, [], 0, 0)
        r, used = _gpu_ept_map(ctx, 0, m[:0], [0x10000])
        assert used == 0
        assert all(np.array_equal(a, b) for a, b in zip(device.read_arenas(ctx, dw), before))
    finally:
        ctx.close()
    w2 = wl("mix2m")   # memslot VM
    ctx = new_ctx()
    try:
        device.load(ctx, w2)
        with pytest.raises(dv.DevirtError):
            _gpu_ept_map(ctx, 0, m, [0x10000])
    finally:
        ctx.close()
