"""GPU path vs the CPU oracle, element by element, through the C ABI.

Bar: bit-exact (everything is integer): translation records, results, the
ordered fault list, every arena byte (A/D bits included) and every pool byte.
"""
import numpy as np
import pytest

import pins
from gpu_util import compare, gpu_batch, log, new_ctx, oracle_batch
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


# ------------------------------------------------------------ golden walks
def _golden_ctx(world):
    import torch
    import paper_1304_3771_amd as dv
    ctx = new_ctx()
    H = pins.H
    o, arena, pool = pins.build_golden(world)
    vm = ctx.vm_create(H(world["arena_bytes"]))
    ctx.vm_write(vm, 0, arena)
    for i, s in enumerate(world["slots"]):
        ctx.memslot_set(vm, i, H(s["gpa"]), H(s["bytes"]), H(s["arena_off"]))
    if "ept_root" in world:
        ctx.vm_set_ept(vm, H(world["ept_root"]))
    asid = ctx.process_create(vm, H(world["cr3"]), world["levels"])
    assert asid == 0
    dpool = torch.from_numpy(pool.copy()).cuda()
    return ctx, vm, o, arena, pool, dpool, dv


@pytest.mark.parametrize("widx", [0, 1, 2, 3, 4])  # 4-level, 5-level, PAE, PAE, 4-level under an EPT
def test_golden_translate(widx):
    import torch
    world = pins.golden_worlds()[widx]
    log(f"golden translate {world['name']}")
    ctx, vm, o, arena, pool, dpool, dv = _golden_ctx(world)
    try:
        for write in (0, 1):
            qs = [q for q in world["queries"]]
            g = torch.from_numpy(np.array([pins.H(q["gva"]) for q in qs], dtype=np.uint64).view(np.int64)).cuda()
            out = torch.zeros(len(qs) * 24, dtype=torch.uint8).cuda()
            ctx.translate(0, g, len(qs), dv.XLAT_WRITE if write else 0, out)
            ctx.sync()
            x = out.cpu().numpy().view(dv.XLAT_DTYPE)
            e = o.translate(0, [pins.H(q["gva"]) for q in qs], dv.XLAT_WRITE if write else 0)
            for i, q in enumerate(qs):
                assert x[i].tobytes() == e[i].tobytes(), (q["gva"], write, x[i], e[i])
                if q["write"] == write:
                    assert (int(x[i]["code"]), int(x[i]["level"]), int(x[i]["gpa"]), int(x[i]["hpa"]),
                            int(x[i]["page_shift"])) == (q["code"], q["level"], pins.H(q["gpa"]), pins.H(q["hpa"]),
                                                         q["shift"])
        # invalid asid
        out = torch.zeros(24, dtype=torch.uint8).cuda()
        g = torch.tensor([0x1000], dtype=torch.int64).cuda()
        ctx.translate(7, g, 1, 0, out)
        ctx.sync()
        x = out.cpu().numpy().view(dv.XLAT_DTYPE)[0]
        assert int(x["code"]) == dv.CODES["INVALID"] and int(x["vm"]) == 0xFFFF
    finally:
        ctx.close()


@pytest.mark.parametrize("widx", [0, 2, 3, 4])  # the worlds with an A/D expectation
def test_golden_set_ad(widx):
    import torch
    world = pins.golden_worlds()[widx]
    ad = world["ad_after_set_ad_write"]
    ctx, vm, o, arena, pool, dpool, dv = _golden_ctx(world)
    try:
        g = torch.tensor([pins.H(ad["gva"])], dtype=torch.int64).cuda()
        out = torch.zeros(24, dtype=torch.uint8).cuda()
        ctx.translate(0, g, 1, dv.XLAT_WRITE | dv.XLAT_SET_AD, out)
        ctx.sync()
        a = np.empty(pins.H(world["arena_bytes"]), np.uint8)
        ctx.vm_read(vm, 0, a)
        o.translate(0, [pins.H(ad["gva"])], dv.XLAT_WRITE | dv.XLAT_SET_AD)
        assert np.array_equal(a, o.arenas[0])
        for e in ad["expect"]:
            assert int.from_bytes(a[pins.H(e["arena_off"]):pins.H(e["arena_off"]) + 8].tobytes(), "little") == \
                pins.H(e["value"])
    finally:
        ctx.close()


@pytest.mark.parametrize("widx", [0, 2, 3, 4])  # the worlds with copies
@pytest.mark.parametrize("path", ["plain", "batch"])
def test_golden_copies(path, widx):
    import torch
    world = pins.golden_worlds()[widx]
    for c in world["copies"]:
        log(f"golden copy {path} {c['gva']} dir {c['dir']}")
        ctx, vm, o, arena, pool, dpool, dv = _golden_ctx(world)
        try:
            H = pins.H
            res = torch.zeros(24, dtype=torch.uint8).cuda()
            if path == "plain":
                f = ctx.copy_to_guest if c["dir"] == 1 else ctx.copy_from_guest
                f(0, H(c["gva"]), dpool.data_ptr(), H(c["len"]), res)
            else:
                req = np.zeros(1, dv.REQUEST_DTYPE)
                req[0] = (H(c["gva"]), dpool.data_ptr(), H(c["len"]), 0, c["dir"], (0, 0, 0), 0)
                dreq = device.upload_requests(req)
                ctx.submit_batch(dreq, 1, res)
            ctx.sync()
            r = res.cpu().numpy().view(dv.RESULT_DTYPE)[0]
            req = np.zeros(1, dv.REQUEST_DTYPE)
            req[0] = (H(c["gva"]), 0, H(c["len"]), 0, c["dir"], (0, 0, 0), 0)
            er = o.copy(req[0])
            assert r.tobytes() == er.tobytes()
            assert (int(r["code"]), int(r["bytes_done"])) == (c["code"], H(c["bytes_done"]))
            a = np.empty(H(world["arena_bytes"]), np.uint8)
            ctx.vm_read(vm, 0, a)
            assert np.array_equal(a, o.arenas[0])
            assert np.array_equal(dpool.cpu().numpy(), o.pool)
        finally:
            ctx.close()


# ------------------------------------------------------------ batches
@pytest.mark.parametrize("name", ["tiny4k", "c1", "mix2m", "multi_vm", "lvl5", "lvl5_1g", "prot", "pae",
                                  "pae_prot", "ept", "ept_faults", "ept_lvl5", "ept_pae", "ept_1g"])
def test_batch_matches_oracle(name):
    w = wl(name)
    log(f"batch {name}: {w.n_requests} requests, {len(w.epoch_end)} epochs")
    got = gpu_batch(w)
    exp = oracle_batch(w)
    assert compare(name, got, exp) == []


# Lengths on both sides of every split in the copy: 16-byte blocks, the 1 KiB
# bound between 16-lane and whole-wavefront segments, and page crossings.
ALIGN_LENS = [1, 2, 15, 16, 17, 31, 100, 255, 256, 257, 511, 1000, 1007, 1008, 1009, 1023, 1024, 1025,
              1100, 2047, 4095, 4096, 4097, 6000]


def _alignment_workload():
    """mix2m's tables with requests at every (guest address mod 16, host address
    mod 16) pair for every length above, alternating direction: one epoch,
    disjoint guest and host ranges laid out through the process's VMAs."""
    import dataclasses
    w = wl("mix2m")
    p = w.procs[0]
    vmas = [(int(b), int(z)) for b, z in p.vmas]
    R = np.zeros(16 * 16 * len(ALIGN_LENS), gen.REQ_DTYPE)
    v, g, h, k = 0, vmas[0][0], 0, 0
    for L in ALIGN_LENS:
        for a in range(16):
            for b in range(16):
                gva = (g + 15) // 16 * 16 + a
                if gva + L > vmas[v][0] + vmas[v][1]:
                    v += 1
                    gva = (vmas[v][0] + 15) // 16 * 16 + a
                host = (h + 15) // 16 * 16 + b
                R[k] = (gva, host, L, p.asid, k % 2, (0, 0, 0), 0)
                g, h, k = gva + L + 48, host + L + 48, k + 1
    return dataclasses.replace(w, requests=R, epoch_end=np.array([k], np.uint64), pool_bytes=h + 64,
                               req_vma=None)


@pytest.mark.parametrize("path", ["batch", "batch_group1", "plain"])
def test_copy_alignments(path):
    """Every source/destination alignment pair and length class, bit-exact."""
    import torch
    import paper_1304_3771_amd as dv
    from oracle import Oracle
    w = _alignment_workload()
    log(f"alignments {path}: {w.n_requests} requests")
    assert Oracle.from_workload(w).check_conflicts(w.requests, w.epoch_end) is None  # one valid epoch
    if path == "plain":
        ctx = new_ctx()
        try:
            dw = device.load(ctx, w)
            n = dw.n
            res = torch.zeros(n * 24, dtype=torch.uint8, device="cuda")
            for i, r in enumerate(dw.reqs_host):
                f = ctx.copy_to_guest if int(r["dir"]) == 1 else ctx.copy_from_guest
                f(int(r["asid"]), int(r["gva"]), int(r["host"]), int(r["len"]), res.data_ptr() + 24 * i)
            ctx.sync()
            got_r = res.cpu().numpy().view(dv.RESULT_DTYPE)
            arenas = device.read_arenas(ctx, dw)
            pool = dw.pool.cpu().numpy()
        finally:
            ctx.close()
        fidx = np.nonzero(got_r["code"] != 0)[0]
        gf = np.zeros(len(fidx), dv.FAULT_DTYPE)
        gf["req_index"], gf["fault_gva"], gf["code"], gf["level"] = fidx, got_r["fault_gva"][fidx], \
            got_r["code"][fidx], got_r["level"][fidx]
        got = (got_r, gf, arenas, pool)
    else:
        got = gpu_batch(w, cfg=dict(group=1) if path == "batch_group1" else None)
    exp = oracle_batch(w)
    assert compare(f"alignments {path}", got, exp) == []
    assert int(np.count_nonzero(exp[0]["bytes_done"])) > w.n_requests // 2  # most requests copy bytes


@pytest.mark.parametrize("cfg", [
    dict(group=1, seg_chunks=1),
    dict(group=64, seg_chunks=64, nontemporal=1),
    dict(group=7, seg_chunks=3, inline_bytes=256, xlat_wg=64, copy_wg=64),
    dict(use_graph=0, copy_wg=1024, copy_wgs_per_cu=1),
])
def test_batch_configs_agree(cfg):
    w = wl("multi_vm")
    log(f"config {cfg}")
    got = gpu_batch(w, cfg=cfg)
    exp = oracle_batch(w)
    assert compare(str(cfg), got, exp) == []


def test_batch_single_epoch_when_conflict_free():
    # C1 has one epoch; run it without the epoch array as well
    w = wl("c1")
    got = gpu_batch(w, epochs=False)
    exp = oracle_batch(w)
    assert compare("c1 no epochs", got, exp) == []


def test_plain_per_request_matches_oracle():
    import torch
    import paper_1304_3771_amd as dv
    w = wl("mix2m")
    log("plain per-request mix2m")
    ctx = new_ctx()
    try:
        dw = device.load(ctx, w)
        n = dw.n
        res = torch.zeros(n * 24, dtype=torch.uint8, device="cuda")
        for i, r in enumerate(dw.reqs_host):
            f = ctx.copy_to_guest if int(r["dir"]) == 1 else ctx.copy_from_guest
            f(int(r["asid"]), int(r["gva"]), int(r["host"]), int(r["len"]), res.data_ptr() + 24 * i)
        ctx.sync()
        got_r = res.cpu().numpy().view(dv.RESULT_DTYPE)
        arenas = device.read_arenas(ctx, dw)
        pool = dw.pool.cpu().numpy()
    finally:
        ctx.close()
    er, ef, ea, ep = oracle_batch(w)
    fidx = np.nonzero(got_r["code"] != 0)[0]
    gf = np.zeros(len(fidx), dv.FAULT_DTYPE)
    gf["req_index"], gf["fault_gva"], gf["code"], gf["level"] = fidx, got_r["fault_gva"][fidx], \
        got_r["code"][fidx], got_r["level"][fidx]
    assert compare("plain", (got_r, gf, arenas, pool), (er, ef, ea, ep)) == []


def test_translate_matches_oracle():
    import torch
    import paper_1304_3771_amd as dv
    from oracle import Oracle
    for name in ("mix2m", "lvl5_1g", "prot", "multi_vm", "pae_prot", "ept_faults", "ept_lvl5", "ept_pae"):
        w = wl(name)
        log(f"translate {name}")
        rng = np.random.default_rng(3)
        ctx = new_ctx()
        try:
            dw = device.load(ctx, w)
            o = Oracle.from_workload(w)
            for p in w.procs[:3]:
                k = min(len(p.leaf_va), 3000)
                sel = rng.choice(len(p.leaf_va), k, replace=False)
                g = p.leaf_va[sel] + rng.integers(0, 4096, k, dtype=np.uint64)
                g = np.concatenate([g, rng.integers(0, 1 << 48, 500, dtype=np.uint64),
                                    p.vmas[:, 0] + p.vmas[:, 1]]).astype(np.uint64)
                for flags in (0, dv.XLAT_WRITE, dv.XLAT_WRITE | dv.XLAT_SET_AD, dv.XLAT_SET_AD):
                    dg = torch.from_numpy(g.view(np.int64)).cuda()
                    out = torch.zeros(len(g) * 24, dtype=torch.uint8, device="cuda")
                    ctx.translate(p.asid, dg, len(g), flags, out)
                    ctx.sync()
                    x = out.cpu().numpy().view(dv.XLAT_DTYPE)
                    e = o.translate(p.asid, g, flags)
                    if not np.array_equal(x.view(np.uint8), e.view(np.uint8)):
                        i = int(np.nonzero((x.view(np.uint8).reshape(-1, 24) != e.view(np.uint8).reshape(-1, 24))
                                           .any(axis=1))[0][0])
                        raise AssertionError(f"{name} asid {p.asid} flags {flags} gva {hex(int(g[i]))}: "
                                             f"gpu {x[i]} oracle {e[i]}")
            arenas = device.read_arenas(ctx, dw)
            for v in range(len(arenas)):
                assert np.array_equal(arenas[v], o.arenas[v]), f"{name}: A/D state differs in vm {v}"
        finally:
            ctx.close()


def test_edge_cases():
    """Empty batch, zero length, bad asid, non-canonical and wrapping ranges,
    a 4 MiB request spanning many passes, requests ending at the user limit."""
    import torch
    import paper_1304_3771_amd as dv
    w = wl("lvl5")
    ctx = new_ctx()
    try:
        dw = device.load(ctx, w)
        # empty batch
        res = torch.zeros(24, dtype=torch.uint8, device="cuda")
        nf = torch.full((1,), 77, dtype=torch.int64, device="cuda")
        ctx.submit_batch(dw.reqs, 0, res, None, None, nf)
        ctx.sync()
        assert int(nf.item()) == 0
        p0 = w.procs[0]
        big = int(p0.vmas[np.argmax(p0.vmas[:, 1]), 0])
        span = int(p0.vmas[:, 1].max())
        # a dedicated 16 MiB host pool: every host range below stays inside it
        hpool = gen.fill_bytes(np.empty(16 << 20, np.uint8), 5, 9)
        epool = torch.from_numpy(hpool.copy()).cuda()
        base = epool.data_ptr()
        edge = [
            (int(p0.leaf_va[0]), base, 0, 0, 1),                       # len 0
            (int(p0.leaf_va[0]), base, 100, 9999, 0),                  # bad asid
            ((1 << 56) - 8, base, 16, 0, 0),                           # runs past the 5-level limit
            ((1 << 64) - 8, base, 16, 0, 1),                           # wraps
            ((1 << 56) - 4096, base, 4096, 0, 0),                      # last user page (unmapped)
            (big + 123, base + 64, min(span - 200, 4 << 20), 0, 0),    # up to 4 MiB, many passes
            (big + 77, base + (8 << 20), min(span - 100, 3 << 20), 0, 1),
        ]
        req = np.zeros(len(edge), dv.REQUEST_DTYPE)
        for i, (g, h, n, a, d) in enumerate(edge):
            req[i] = (g, h, n, a, d, (0, 0, 0), 0)
        hreq = req.copy()
        hreq["host"] -= np.uint64(base)
        dreq = device.upload_requests(req)
        res = torch.zeros(len(edge) * 24, dtype=torch.uint8, device="cuda")
        faults = torch.zeros(len(edge) * 24, dtype=torch.uint8, device="cuda")
        nf = torch.zeros(1, dtype=torch.int64, device="cuda")
        ctx.submit_batch(dreq, len(edge), res, [len(edge) - 1, len(edge)], faults, nf)
        ctx.sync()
        r = res.cpu().numpy().view(dv.RESULT_DTYPE)
        assert all(h - base + n <= hpool.size for (g, h, n, a, d) in edge)
        from oracle import Oracle
        o = Oracle.from_workload(w, pool=hpool.copy())
        er, ef = o.batch(hreq)
        assert np.array_equal(r.view(np.uint8), er.view(np.uint8)), (r, er)
        k = int(nf.item())
        assert np.array_equal(faults.cpu().numpy()[:24 * k].view(dv.FAULT_DTYPE).view(np.uint8), ef.view(np.uint8))
        assert np.array_equal(epool.cpu().numpy(), o.pool)
        for v, a in enumerate(device.read_arenas(ctx, dw)):
            assert np.array_equal(a, o.arenas[v])
        # API misuse is an error, not a fault
        with pytest.raises(dv.DevirtError):
            ctx.submit_batch(dreq, len(edge), res, [3, 2, len(edge)])
        with pytest.raises(dv.DevirtError):
            ctx.memslot_set(0, 0, 4096, 4096 * 3, 1)
        with pytest.raises(dv.DevirtError):
            ctx.set_config(group=0)
    finally:
        ctx.close()


def test_queue_overflow_copies_inline(monkeypatch):
    """With a tiny segment queue the translating wavefronts copy the rest themselves."""
    monkeypatch.setenv("DEVIRT_SEG_CAP", "64")
    w = wl("mix2m")
    got = gpu_batch(w)
    exp = oracle_batch(w)
    assert compare("overflow", got, exp) == []


def _cross_epoch_reuse(w):
    """Pairs of consecutive epochs whose requests share guest bytes (same process)
    and whose host ranges overlap."""
    r = w.requests
    ep = np.repeat(np.arange(len(w.epoch_end)), np.diff(np.concatenate([[0], w.epoch_end.astype(np.int64)])))
    guest = host = 0
    for e in range(len(w.epoch_end) - 1):
        a, b = r[ep == e], r[ep == e + 1]
        for x, y, key in ((a, b, "gva"), (a, b, "host")):
            lo = np.sort(x[key])
            hi = (x[key] + x["len"].astype(np.uint64))[np.argsort(x[key])]
            for q in y[:200]:
                j = np.searchsorted(lo, q[key] + np.uint64(q["len"])) - 1
                if j >= 0 and np.any(hi[:j + 1] > q[key]):
                    if key == "host":
                        host += 1
                    elif np.any(x["asid"][np.argsort(x[key])][:j + 1][hi[:j + 1] > q[key]] == q["asid"]):
                        guest += 1
                    break
    return guest, host


@pytest.mark.parametrize("overlap,spill_side", [(1, 1), (1, 0), (0, 1)])
def test_overflow_across_epochs(monkeypatch, overlap, spill_side):
    """Many epochs that reuse guest and host bytes, a segment queue of 64
    (one segment per queue part and half), inline copies of runs up to 256 B:
    with translation overlapped (the next epoch is translated while the
    previous one is copied) no translating wavefront may move payload bytes,
    so inline copies are off after the first epoch and overflowing groups are
    copied by the spill pass; without overlap the translating wavefronts copy
    them in place.  Bit-exact on results, faults, every arena and pool byte,
    with graphs, and again with device counters that show both paths ran."""
    import torch
    monkeypatch.setenv("DEVIRT_SEG_CAP", "64")
    w = wl("epochs")
    assert len(w.epoch_end) >= 8
    g, h = _cross_epoch_reuse(w)
    assert g > 0 and h > 0, (g, h)
    cfg = dict(inline_bytes=256, overlap=overlap, group=8, spill_side=spill_side)
    exp = oracle_batch(w)
    got = gpu_batch(w, cfg=cfg)
    assert compare(f"epochs overlap={overlap}", got, exp) == []
    got = gpu_batch(w, cfg=cfg, t_done=True)
    assert compare(f"epochs overlap={overlap} t_done", got, exp) == []
    assert np.all(got[4]["t_done"] > 0)
    ctx = new_ctx(**cfg)
    try:
        ctx.set_profiling(True, counters=True)
        got = gpu_batch(w, ctx=ctx)
        st = got[4]["stats"]
    finally:
        ctx.close()
    assert compare(f"epochs overlap={overlap} counters", got, exp) == []
    log(f"overlap={overlap}: {st['spilled_groups']} groups spilled, {st['inline_segments']} runs copied "
        f"by translating wavefronts, {st['segments']} queued")
    assert st["inline_segments"] > 0
    if overlap:
        assert st["spilled_groups"] > 0
    else:
        assert st["spilled_groups"] == 0


@pytest.mark.parametrize("spill_side", [1, 0])
def test_spill_passes_with_empty_epochs(monkeypatch, spill_side):
    """The spill pass of an epoch runs on the translate stream, beside the
    epoch's own copy and ahead of the next epoch's translation (spill_side 1),
    or on the copy stream right after the epoch's copy (0).  Empty epochs
    (every boundary given twice, and an empty first and last epoch) leave
    some epochs without a translation or copy of their own.  With a
    64-segment queue, so that groups do spill, and overlap on: results,
    faults, every arena and pool byte equal the oracle, with completion
    times, with device counters showing spills, and over three graph replays
    of the batch (the oracle applies it three times)."""
    import dataclasses
    from oracle import Oracle
    monkeypatch.setenv("DEVIRT_SEG_CAP", "64")
    w = wl("epochs")
    ends = w.epoch_end.astype(np.uint64)
    ep = np.concatenate([[0], np.repeat(ends, 2), [ends[-1]]]).astype(np.uint64)
    w2 = dataclasses.replace(w, epoch_end=ep)
    assert np.sum(np.diff(np.concatenate([[0], ep.astype(np.int64)])) == 0) >= len(ends) + 1
    exp = oracle_batch(w)
    cfg = dict(overlap=1, group=8, spill_side=spill_side)
    assert compare("empty epochs", gpu_batch(w2, cfg=cfg), exp) == []
    got = gpu_batch(w2, cfg=cfg, t_done=True)
    assert compare("empty epochs t_done", got, exp) == []
    assert np.all(got[4]["t_done"] > 0)
    ctx = new_ctx(**cfg)
    try:
        ctx.set_profiling(True, counters=True)
        got = gpu_batch(w2, ctx=ctx)
        st = got[4]["stats"]
    finally:
        ctx.close()
    assert compare("empty epochs counters", got, exp) == []
    assert st["spilled_groups"] > 0, st
    o = Oracle.from_workload(w)
    for _ in range(3):
        er, ef = o.batch(w.requests)
    assert compare("empty epochs, 3 replays", gpu_batch(w2, cfg=cfg, repeat=3), (er, ef, o.arenas, o.pool)) == []


def test_maximum_length_requests():
    """Requests of the largest length a descriptor holds (2^32 - 1 bytes) in a
    6 GiB guest with one fully mapped 4.8 GiB region: a read and a write of
    the whole length at unaligned guest and host addresses, and a read that
    runs off the mapped part of the region 2 GiB in, which copies exactly up
    to its first unmapped page; each in its own epoch.  Results, faults,
    every arena byte and every pool byte against the oracle, with the
    benchmark's launch configuration and with the workgroup walk of large
    requests."""
    import dataclasses
    GiB = 1 << 30
    sp = gen.spec("C2").replace(name="maxlen", mem_bytes=6 * GiB, p_np=0.0, vmas_per_proc=1, mapped_frac=0.8,
                                n_requests=16, seed=77)
    w = gen.make_workload(sp)
    p = w.procs[0]
    b, z = (int(x) for x in p.vmas[0])
    L = (1 << 32) - 1
    assert z >= L + 8192
    R = np.zeros(3, gen.REQ_DTYPE)
    R[0] = (b + 123, 0, L, p.asid, 0, (0, 0, 0), 0)                     # guest -> host
    R[1] = (b + 4096 + 77, L + 69, L, p.asid, 1, (0, 0, 0), 0)          # host -> guest
    R[2] = (b + z - (2 << 30) + 9, 5, L, p.asid, 0, (0, 0, 0), 0)       # off the mapped part
    w2 = dataclasses.replace(w, requests=R, epoch_end=np.array([1, 2, 3], np.uint64), pool_bytes=2 * L + 256,
                             req_vma=None)
    exp = oracle_batch(w2)
    er = exp[0]
    assert np.all(er["bytes_done"][:2] == L) and er["code"][2] != 0 and er["bytes_done"][2] > GiB
    log(f"max length: {L} bytes; the third request stops after {int(er['bytes_done'][2])}")
    for cfg in (dict(group=64, seg_chunks=1, xlat_wgs_per_cu=2, copy_wg=1024, copy_wgs_per_cu=16, overlap=1),
                dict(large_pages=256, overlap=1)):
        assert compare(f"max length {cfg}", gpu_batch(w2, cfg=cfg), exp) == []


def test_completion_times_and_repeat():
    w = wl("multi_vm")
    got = gpu_batch(w, t_done=True)
    exp = oracle_batch(w)
    assert compare("t_done", got, exp) == []
    td = got[4]["t_done"]
    assert np.all(td > 0) and np.all(td < 60e9)


@pytest.mark.parametrize("overlap", [0, 1])
def test_large_requests_by_workgroups(monkeypatch, overlap):
    """Requests of more than large_pages pages are walked by the four
    wavefronts of a workgroup together, round by round, agreeing on each
    request's first faulting page before any A/D bit or copy.  Bit-exact
    against the oracle with the smallest threshold, with completion times,
    and with a 64-segment queue (overflowing large requests are copied by
    their own wavefronts, or with overlap go to the spill pass alone)."""
    import paper_1304_3771_amd as dv
    w = wl("large")
    pages = ((w.requests["gva"] + w.requests["len"] - 1) >> 12) - (w.requests["gva"] >> 12) + 1
    n_large = int(np.count_nonzero((w.requests["len"] > 0) & (pages > 64)))
    exp = oracle_batch(w)
    faulted_large = int(np.count_nonzero((pages > 64) & (exp[0]["code"] != 0) & (exp[0]["bytes_done"] > 4096)))
    log(f"large: {w.n_requests} requests, {n_large} of more than 64 pages ({faulted_large} fault past their "
        f"first page), {len(w.epoch_end)} epochs")
    assert n_large > 50 and faulted_large > 5
    cfg = dict(large_pages=64, overlap=overlap, group=8)
    got = gpu_batch(w, cfg=cfg, t_done=True)
    assert compare(f"large overlap={overlap}", got, exp) == []
    td = got[4]["t_done"]
    assert np.all(td > 0) and np.all(td < 60e9)
    # device counters: every large request went through the workgroup walk
    ctx = new_ctx(**cfg)
    try:
        ctx.set_profiling(True, counters=True)
        ctx.reset_stats()
        got = gpu_batch(w, ctx=ctx)
        st = ctx.get_stats()
    finally:
        ctx.close()
    assert compare(f"large overlap={overlap} counters", got, exp) == []
    assert st["large_requests"] == n_large, (st["large_requests"], n_large)
    monkeypatch.setenv("DEVIRT_SEG_CAP", "64")
    ctx = new_ctx(**cfg)
    try:
        ctx.set_profiling(True, counters=True)
        ctx.reset_stats()
        got = gpu_batch(w, ctx=ctx)
        st = ctx.get_stats()
    finally:
        ctx.close()
    log(f"large, 64-segment queue, overlap={overlap}: {st['spilled_groups']} spilled, "
        f"{st['inline_segments']} runs copied by translating wavefronts")
    assert compare(f"large overlap={overlap} tiny queue", got, exp) == []
    if overlap:
        assert st["spilled_groups"] > 0
    else:
        assert st["inline_segments"] > 0
