"""Serving loop: every operation's result, and all memory, are the same alone
(one operation at a time through the plain per-request path) and in the mix
(continuous batching over several streams, each completion mode), and both
equal the oracle.  Tolerance: none (bit-exact).  Device-side batch windows
show that batches of the non-blocking modes ran on the GPU at the same time,
and that the blocking mode ran one at a time."""
import time

import numpy as np
import pytest

from gpu_util import log, new_ctx
from oracle import Oracle
from workload import device, gen

pytestmark = pytest.mark.gpu

MiB = 1 << 20
CLASSES = ((0.60, "uniform", 24, 24, 1), (0.25, "uniform", 4096, 4096, 0),
           (0.14, "loguniform", 16 << 10, 256 << 10, 0), (0.01, "uniform", 1 << 20, 1 << 20, 1))


@pytest.fixture(scope="module", params=["memslots", "ept", "c4"])
def trace(request):
    """Two VMs translated through their memslots, or through EPTs with some
    leaves not present, read-only or misconfigured (256 MiB each, 1 MiB
    frames); or two of the serving configuration's VMs at its own shape (4 GiB
    each, 4 processes, 16 memslots, 6 MiB thread windows) with its own class
    mix, 4,147,200-byte camera frames included."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if request.param == "c4":
        wl = gen.make_workload(gen.spec("C4", n_vms=2, seed=46), requests=False)
        tr = gen.make_serving_trace(wl, 3000, 2e5, threads_per_proc=8, classes=gen.C4_CLASSES,
                                    host_mode="unique", seed=47)
        assert np.count_nonzero(tr.requests["len"] == 4147200) >= 10
        return wl, tr
    sp = gen.spec("C4", n_vms=2, procs_per_vm=2, mem_bytes=256 * MiB, seed=44)
    if request.param == "ept":
        sp = sp.replace(ept=True, ept_np=0.02, ept_ro=0.03, ept_mis=0.01)
    wl = gen.make_workload(sp, requests=False)
    tr = gen.make_serving_trace(wl, 3000, 2e5, threads_per_proc=8, window=2 * MiB, classes=CLASSES,
                                host_mode="unique", seed=45)
    return wl, tr


@pytest.fixture(scope="module")
def expected(trace):
    """The oracle applied to the operations in submission order."""
    wl, tr = trace
    arenas = [wl.arena_image(v) for v in range(len(wl.vms))]
    opool = gen.fill_bytes(np.empty(tr.pool_bytes, np.uint8), wl.seed, gen.POOL_KEY)
    o = Oracle(arenas, [v.slots for v in wl.vms], [(p.vm, p.cr3, p.levels) for p in wl.procs], opool,
               ept=[v.ept_root for v in wl.vms])
    er, _ = o.batch(tr.requests)
    return er, o.arenas, o.pool


def _load(ctx, wl, tr):
    import torch
    dw = device.load(ctx, wl)
    pool = torch.from_numpy(gen.fill_bytes(np.empty(tr.pool_bytes, np.uint8), wl.seed, gen.POOL_KEY)).cuda()
    reqs = tr.requests.copy()
    reqs["host"] += np.uint64(pool.data_ptr())
    return dw, pool, reqs


@pytest.fixture(scope="module")
def alone(trace):
    """Every operation alone: one at a time, in submission order, through the
    plain per-request path."""
    import torch
    import paper_1304_3771_amd as dv
    wl, tr = trace
    n = len(tr.requests)
    log("serving: alone")
    ctx = new_ctx()
    try:
        dw, pool, reqs = _load(ctx, wl, tr)
        res = torch.zeros(n * 24, dtype=torch.uint8, device="cuda")
        stream = torch.cuda.current_stream()
        for i, r in enumerate(reqs):
            f = ctx.copy_to_guest if int(r["dir"]) == 1 else ctx.copy_from_guest
            f(int(r["asid"]), int(r["gva"]), int(r["host"]), int(r["len"]), res.data_ptr() + 24 * i, stream)
            stream.synchronize()
        return (res.cpu().numpy().view(dv.RESULT_DTYPE).copy(), device.read_arenas(ctx, dw),
                pool.cpu().numpy())
    finally:
        ctx.close()


def _overlapping_windows(c):
    """Pairs of distinct batches whose device windows overlap."""
    w = np.unique(np.stack([c["dev_start_ns"], c["dev_end_ns"]], axis=1), axis=0)
    w = w[np.argsort(w[:, 0], kind="stable")]
    pairs = 0
    ends = []  # ends of the windows still open at the current start
    for a, b in w:
        ends = [e for e in ends if e > a]
        pairs += len(ends)
        ends.append(b)
    return pairs, len(w)


@pytest.mark.parametrize("completion", ["poll", "notify", "blocking"])
def test_alone_vs_mix(trace, alone, expected, completion):
    wl, tr = trace
    n = len(tr.requests)
    alone_res, alone_arenas, alone_pool = alone
    # in the mix: Poisson arrivals replayed in bursts into the serving loop
    log(f"serving: mix, completion by {completion}")
    ctx = new_ctx()
    try:
        dw, pool, reqs = _load(ctx, wl, tr)
        budget = max(4 * MiB, int(tr.requests["len"].max()))
        srv = ctx.server_start(max_inflight=256, pool_bytes=budget, max_batch=64, streams=3,
                               completion=completion, device_times=True)
        comps = []
        try:
            t0 = time.monotonic_ns()
            i = 0
            while i < n:
                now = time.monotonic_ns() - t0
                j = int(np.searchsorted(tr.arrival_ns, now, side="right"))
                j = max(j, i + 1)
                srv.submit(reqs[i:j])
                i = j
                comps.append(srv.poll())
            srv.drain()
            comps.append(srv.poll(n))
            st = srv.stats()
        finally:
            srv.stop()
        # both launch kinds ran: small batches as one direct kernel, the rest queued
        assert 0 < st["direct_launches"] < st["launches"], st
        c = np.concatenate(comps)
        assert len(c) == n and np.array_equal(np.sort(c["ticket"]), np.arange(n))
        c = c[np.argsort(c["ticket"])]
        mix_arenas = device.read_arenas(ctx, dw)
        mix_pool = pool.cpu().numpy()
    finally:
        ctx.close()
    for f in ("bytes_done", "fault_gva", "code", "level"):
        assert np.array_equal(c[f], alone_res[f]), f
    for a, b in zip(mix_arenas, alone_arenas):
        assert np.array_equal(a, b)
    assert np.array_equal(mix_pool, alone_pool)
    # batches on the device: windows from timing events around each launch
    assert np.all(c["dev_end_ns"] > c["dev_start_ns"])
    pairs, batches = _overlapping_windows(c)
    log(f"serving {completion}: {batches} batches, {pairs} pairs ran on the GPU at the same time")
    if completion == "blocking":
        assert pairs == 0, "blocking mode ran two batches at once"
    else:
        assert pairs > 0, "no two batches were on the GPU at the same time"
    # one operation in flight per guest thread; admitted ones overlap in time
    key = reqs["asid"].astype(np.uint64) << np.uint64(32) | reqs["tag"].astype(np.uint64)
    for k in np.unique(key):
        idx = np.nonzero(key == k)[0]
        assert np.all(c["t_admit_ns"][idx[1:]] >= c["t_done_ns"][idx[:-1]]), "two ops of one thread overlapped"
    # the byte budget: at every admission the admitted-and-unfinished bytes fit the pool
    ev = sorted([(int(t), 1, int(b)) for t, b in zip(c["t_admit_ns"], reqs["len"])] +
                [(int(t), 0, -int(b)) for t, b in zip(c["t_done_ns"], reqs["len"])])
    cur = peak = 0
    for t, kind, b in ev:
        cur += b
        peak = max(peak, cur)
    assert peak <= budget or peak <= int(reqs["len"].max())
    # both equal the oracle applied in submission order
    er, oarenas, opool = expected
    for f in ("bytes_done", "fault_gva", "code", "level"):
        assert np.array_equal(c[f], er[f]), f
    for a, b in zip(mix_arenas, oarenas):
        assert np.array_equal(a, b)
    assert np.array_equal(mix_pool, opool)


def test_server_refuses_misuse(trace):
    import paper_1304_3771_amd as dv
    wl, tr = trace
    ctx = new_ctx()
    try:
        with pytest.raises(dv.DevirtError):
            ctx.server_start(max_inflight=0)
        import ctypes
        bad = dv.devirt.ServerCfg(16, MiB, 0, 2, 3)  # no such completion mode
        h = ctypes.c_void_p()
        assert dv.lib().devirt_server_start(ctx._h, ctypes.byref(bad), ctypes.byref(h)) == -22
        srv = ctx.server_start(max_inflight=16, pool_bytes=MiB, streams=2)
        try:
            with pytest.raises(dv.DevirtError):   # the server owns the context
                ctx.vm_create(1 << 20)
        finally:
            srv.stop()
        ctx.vm_create(1 << 20)                     # usable again after stop
    finally:
        ctx.close()


@pytest.mark.parametrize("kind", ["memslots", "ept"])
def test_map_batches_in_thread_order(kind):
    """A guest thread's map batch (section 4.2: the backend maps pages into the
    process between forwarded copies) runs in the thread's order: a copy into
    a region nothing maps faults, the map batch maps it, and the next copies
    into and out of it succeed.  Meanwhile the other threads' operations keep
    arriving.  Every copy's result, every map's result, the map batch's
    summary, guest memory and host bytes equal the oracle applied in
    submission order."""
    import torch
    import pins
    from oracle.oracle import MAP_DTYPE
    sp = gen.spec("C4", n_vms=2, procs_per_vm=2, mem_bytes=256 * MiB, seed=48)
    if kind == "ept":
        sp = sp.replace(ept=True, ept_np=0.02, ept_ro=0.03, ept_mis=0.01)
    wl = gen.make_workload(sp, requests=False)
    tr = gen.make_serving_trace(wl, 1600, 2e5, threads_per_proc=8, window=2 * MiB, classes=CLASSES,
                                host_mode="unique", seed=49)
    p = wl.procs[1]
    base = 0x7E00_0000_0000            # a region no VMA of the process covers
    assert all(not (int(b) <= base < int(b) + int(s)) for b, s in p.vmas)
    rng = np.random.default_rng(50)
    fr = pins.usable_frames(wl, p.vm, pins.free_frames(wl, p.vm, 400, rng))
    assert len(fr) >= 40
    npg = 8
    maps = np.zeros(npg + 1, MAP_DTYPE)
    maps["gva"][:npg] = base + 4096 * np.arange(npg, dtype=np.uint64)
    maps["gpa"][:npg] = fr[:npg]
    maps["flags"][:npg] = 1                                   # writable
    maps[npg] = (1 << 47, int(fr[npg]), 1, 0)   # non-canonical: fails
    pool = [int(f) for f in fr[npg + 1:]]
    # the thread's operations (a tag no trace thread has), host bytes after the trace's
    extra = 64 << 10
    h0 = tr.pool_bytes
    mine = np.zeros(3, tr.requests.dtype)
    mine["asid"], mine["tag"] = p.asid, 999
    mine["gva"] = base + 100
    mine["len"] = (12000, 20000, 20000)
    mine["dir"] = (1, 1, 0)
    mine["host"] = (h0, h0, h0 + 32768)
    # submission order: trace[:a], mine[0], trace[a:b], the map, trace[b:c], mine[1:3], trace[c:]
    n = len(tr.requests)
    a, b, c = n // 4, n // 2, 3 * n // 4
    hbytes = gen.fill_bytes(np.empty(tr.pool_bytes + extra, np.uint8), wl.seed, gen.POOL_KEY)
    arenas = [wl.arena_image(v) for v in range(len(wl.vms))]
    o = Oracle(arenas, [v.slots for v in wl.vms], [(q.vm, q.cr3, q.levels) for q in wl.procs], hbytes.copy(),
               ept=[v.ept_root for v in wl.vms])
    e = [o.batch(tr.requests[:a])[0], o.batch(mine[0:1])[0], o.batch(tr.requests[a:b])[0]]
    em, eused = o.map_pages(p.asid, maps, pool)
    e += [o.batch(tr.requests[b:c])[0], o.batch(mine[1:3])[0], o.batch(tr.requests[c:])[0]]
    assert e[1]["code"][0] != 0 and np.all(e[4]["code"] == 0) and eused > 0
    assert np.all(em["code"][:npg] == 0) and em["code"][npg] != 0
    log(f"serving maps {kind}")
    ctx = new_ctx()
    try:
        dw = device.load(ctx, wl)
        hb = torch.from_numpy(hbytes.copy()).cuda()
        reqs = tr.requests.copy()
        reqs["host"] += np.uint64(hb.data_ptr())
        mreqs = mine.copy()
        mreqs["host"] += np.uint64(hb.data_ptr())
        srv = ctx.server_start(max_inflight=128, pool_bytes=4 * MiB, max_batch=32, streams=3)
        comps = []
        try:
            import paper_1304_3771_amd as dv
            with pytest.raises(dv.DevirtError):     # refused at submission, no ticket taken
                srv.submit_map(p.asid, 999, maps, [pool[0] + 8])
            for part in (reqs[:a], mreqs[0:1], reqs[a:b], None, reqs[b:c], mreqs[1:3], reqs[c:]):
                if part is None:
                    t_map, mres = srv.submit_map(p.asid, 999, maps, pool)
                else:
                    for k in range(0, len(part), 100):   # in bursts, completions taken between
                        assert srv.submit(part[k:k + 100]) == len(part[k:k + 100])
                        comps.append(srv.poll())
            srv.drain()
            comps.append(srv.poll(n + 8))
        finally:
            srv.stop()
        got = np.concatenate(comps)
        assert len(got) == n + 4 and np.array_equal(np.sort(got["ticket"]), np.arange(n + 4))
        got = got[np.argsort(got["ticket"])]
        garenas = device.read_arenas(ctx, dw)
        ghost = hb.cpu().numpy()
    finally:
        ctx.close()
    assert t_map == b + 1
    # the results in submission order, the map batch's summary in its place
    order = np.r_[0:a, a, a + 1:b + 1, b + 2:c + 2, c + 2, c + 3, c + 4:n + 4]
    want = np.concatenate(e[:3] + e[3:])
    for f in ("bytes_done", "fault_gva", "code", "level"):
        assert np.array_equal(got[f][order], want[f]), f
    s = got[t_map]
    assert int(s["bytes_done"]) == 4096 * npg
    assert (int(s["code"]), int(s["level"]), int(s["fault_gva"])) == \
        (int(em["code"][npg]), int(em["level"][npg]), int(em["fault_gva"][npg]))
    assert mres.tobytes() == em.tobytes()
    for x, y in zip(garenas, o.arenas):
        assert np.array_equal(x, y)
    assert np.array_equal(ghost, o.pool)
    # the thread's operations, the map batch included, ran one after another
    mine_t = [a, t_map, c + 2, c + 3]
    assert np.all(got["t_admit_ns"][mine_t[1:]] >= got["t_done_ns"][mine_t[:-1]])


def test_ept_map_batches_in_thread_order():
    """Both halves of mapping a page in a VM with an EPT (section 4.2), as one
    guest thread's operations in the serving loop: a copy into an unmapped
    region faults in the guest's tables; a guest-table map batch points the
    region at guest-physical pages far above guest memory; the next copy
    faults in the EPT; an EPT map batch backs those pages with free arena
    pages; the copies after it succeed.  Other threads' operations keep
    arriving meanwhile.  Every result, both batches' summaries and per-map
    results, guest memory and host bytes equal the oracle applied in
    submission order."""
    import torch
    import pins
    import paper_1304_3771_amd as dv
    from oracle.oracle import EPT_MAP_DTYPE, MAP_DTYPE
    sp = gen.spec("C4", n_vms=2, procs_per_vm=2, mem_bytes=256 * MiB, seed=52)
    sp = sp.replace(ept=True, ept_np=0.02, ept_ro=0.03, ept_mis=0.01)
    wl = gen.make_workload(sp, requests=False)
    tr = gen.make_serving_trace(wl, 1600, 2e5, threads_per_proc=8, window=2 * MiB, classes=CLASSES,
                                host_mode="unique", seed=53)
    p = wl.procs[2]
    v = wl.vms[p.vm]
    base = 0x7E00_0000_0000
    assert all(not (int(b) <= base < int(b) + int(s)) for b, s in p.vmas)
    rng = np.random.default_rng(54)
    fr = pins.usable_frames(wl, p.vm, pins.free_frames(wl, p.vm, 600, rng))
    npg = 8
    far = np.uint64(1 << 40) + np.uint64(4096) * np.arange(npg, dtype=np.uint64)
    gmaps = np.zeros(npg, MAP_DTYPE)
    gmaps["gva"] = base + 4096 * np.arange(npg, dtype=np.uint64)
    gmaps["gpa"] = far
    gmaps["flags"] = 1
    gpool = [int(f) for f in fr[:200]]
    emaps = np.zeros(npg + 1, EPT_MAP_DTYPE)
    emaps["gpa"][:npg] = far
    emaps["hpa"][:npg] = gen.gpa_to_arena(v.slots, fr[200:200 + npg])
    emaps["flags"][:npg] = 7
    emaps[npg] = (int(far[0]) + (1 << 48), int(emaps["hpa"][0]), 7, 0)   # past the EPT's reach: fails
    epool = [int(x) for x in gen.gpa_to_arena(v.slots, fr[300:340])]
    extra = 64 << 10
    h0 = tr.pool_bytes
    mine = np.zeros(4, tr.requests.dtype)
    mine["asid"], mine["tag"] = p.asid, 999
    mine["gva"] = base + 100
    mine["len"] = (12000, 12000, 20000, 20000)
    mine["dir"] = (1, 1, 1, 0)
    mine["host"] = (h0, h0, h0, h0 + 32768)
    n = len(tr.requests)
    cut = [n // 5, 2 * n // 5, 3 * n // 5, 4 * n // 5]
    hbytes = gen.fill_bytes(np.empty(tr.pool_bytes + extra, np.uint8), wl.seed, gen.POOL_KEY)
    arenas = [wl.arena_image(k) for k in range(len(wl.vms))]
    o = Oracle(arenas, [x.slots for x in wl.vms], [(q.vm, q.cr3, q.levels) for q in wl.procs], hbytes.copy(),
               ept=[x.ept_root for x in wl.vms])
    # submission order: T0 c0 T1 gmap T2 c1 T3 emap T4 c2 c3
    R = tr.requests
    want = [o.batch(R[:cut[0]])[0], o.batch(mine[0:1])[0], o.batch(R[cut[0]:cut[1]])[0]]
    eg, egu = o.map_pages(p.asid, gmaps, gpool)
    want += [o.batch(R[cut[1]:cut[2]])[0], o.batch(mine[1:2])[0], o.batch(R[cut[2]:cut[3]])[0]]
    ee, eeu = o.ept_map_pages(p.vm, emaps, epool)
    want += [o.batch(R[cut[3]:])[0], o.batch(mine[2:4])[0]]
    assert want[1]["code"][0] != 0 and want[4]["code"][0] != 0 and np.all(want[7]["code"] == 0)
    assert want[1]["code"][0] != want[4]["code"][0]          # a guest-table fault, then an EPT fault
    assert np.all(eg["code"] == 0) and np.all(ee["code"][:npg] == 0) and ee["code"][npg] != 0 and eeu > 0
    log("serving: guest-table and EPT maps in a thread's order")
    ctx = new_ctx()
    try:
        dw = device.load(ctx, wl)
        hb = torch.from_numpy(hbytes.copy()).cuda()
        reqs = R.copy()
        reqs["host"] += np.uint64(hb.data_ptr())
        mreqs = mine.copy()
        mreqs["host"] += np.uint64(hb.data_ptr())
        srv = ctx.server_start(max_inflight=128, pool_bytes=4 * MiB, max_batch=32, streams=3)
        comps = []
        try:
            with pytest.raises(dv.DevirtError):     # an unknown VM, refused at submission
                srv.submit_ept_map(p.asid, 999, len(wl.vms), emaps, epool)
            with pytest.raises(dv.DevirtError):     # a pool page outside the arena
                srv.submit_ept_map(p.asid, 999, p.vm, emaps, [v.arena_bytes])
            tick = {}
            parts = [("T", reqs[:cut[0]]), ("C", mreqs[0:1]), ("T", reqs[cut[0]:cut[1]]), ("G", None),
                     ("T", reqs[cut[1]:cut[2]]), ("C", mreqs[1:2]), ("T", reqs[cut[2]:cut[3]]), ("E", None),
                     ("T", reqs[cut[3]:]), ("C", mreqs[2:4])]
            for kind, part in parts:
                if kind == "G":
                    tick["g"], gres = srv.submit_map(p.asid, 999, gmaps, gpool)
                elif kind == "E":
                    tick["e"], eres = srv.submit_ept_map(p.asid, 999, p.vm, emaps, epool)
                else:
                    for k in range(0, len(part), 100):
                        assert srv.submit(part[k:k + 100]) == len(part[k:k + 100])
                        comps.append(srv.poll())
            srv.drain()
            comps.append(srv.poll(n + 8))
        finally:
            srv.stop()
        got = np.concatenate(comps)
        assert len(got) == n + 6 and np.array_equal(np.sort(got["ticket"]), np.arange(n + 6))
        got = got[np.argsort(got["ticket"])]
        garenas = device.read_arenas(ctx, dw)
        ghost = hb.cpu().numpy()
    finally:
        ctx.close()
    is_map = np.zeros(n + 6, bool)
    is_map[[tick["g"], tick["e"]]] = True
    w = np.concatenate(want)
    for f in ("bytes_done", "fault_gva", "code", "level"):
        assert np.array_equal(got[f][~is_map], w[f]), f
    for t, er, res in ((tick["g"], eg, gres), (tick["e"], ee, eres)):
        assert res.tobytes() == er.tobytes()
        ok = er["code"] == 0
        assert int(got["bytes_done"][t]) == 4096 * int(ok.sum())
        first = np.nonzero(~ok)[0]
        want_sum = (0, 0, 0) if not len(first) else \
            (int(er["code"][first[0]]), int(er["level"][first[0]]), int(er["fault_gva"][first[0]]))
        assert (int(got["code"][t]), int(got["level"][t]), int(got["fault_gva"][t])) == want_sum
    for x, y in zip(garenas, o.arenas):
        assert np.array_equal(x, y)
    assert np.array_equal(ghost, o.pool)
    mine_t = np.nonzero(np.concatenate([np.zeros(len(a), bool) if i not in (1, 4, 7) else np.ones(len(a), bool)
                                        for i, a in enumerate(want)]))[0]
    seq = sorted(list(np.nonzero(~is_map)[0][mine_t]) + [tick["g"], tick["e"]])
    assert np.all(got["t_admit_ns"][seq[1:]] >= got["t_done_ns"][seq[:-1]])
