"""The CPU oracle against facts other than itself (hand-derived walks,
the generator's encoded map, per-byte brute force, memcpy, invariants)."""
import pytest

import pins
from workload import gen

SPECS = pins.small_specs()
_WL = {}


def wl(name):
    if name not in _WL:
        _WL[name] = gen.make_workload(SPECS[name])
    return _WL[name]


def test_golden_walks_ad_and_copies():
    assert pins.check_golden() == []


def test_golden_maps():
    assert pins.check_golden_maps() == []


def test_golden_ept_maps():
    assert pins.check_golden_ept_maps() == []


@pytest.mark.parametrize("name", ["ept", "ept_faults", "ept_lvl5", "ept_pae", "ept_1g"])
def test_ept_map_properties(name):
    assert pins.check_ept_map_properties(wl(name)) == []


def test_golden_fifo_cache():
    assert pins.check_golden_fifo() == []


@pytest.mark.parametrize("name", ["c1", "mix2m", "multi_vm", "prot", "pae_prot", "ept_faults"])
def test_fifo_cache_properties(name):
    assert pins.check_fifo_properties(wl(name)) == []


# worlds whose encoded tables are all reachable (no not-present upper entries)
@pytest.mark.parametrize("name", ["c1", "mix2m", "lvl5", "lvl5_1g", "pae"])
def test_map_properties(name):
    assert pins.check_map_properties(wl(name)) == []


@pytest.mark.parametrize("name", ["tiny4k", "c1", "mix2m", "multi_vm", "lvl5", "lvl5_1g", "pae"])
def test_encode_decode_roundtrip(name):
    assert pins.check_roundtrip(wl(name)) == []


@pytest.mark.parametrize("name", ["tiny4k", "c1", "mix2m", "multi_vm", "lvl5", "lvl5_1g", "prot", "pae",
                                  "pae_prot"])
def test_per_byte_bruteforce(name):
    assert pins.check_bruteforce(wl(name), max_requests=120) == []


def test_identity_tables_equal_memcpy():
    assert pins.check_identity() == []


@pytest.mark.parametrize("name", ["c1", "mix2m", "multi_vm", "lvl5", "prot", "pae", "pae_prot"])
def test_ad_closed_form(name):
    assert pins.check_ad_closed_form(wl(name)) == []


@pytest.mark.parametrize("name", ["tiny4k", "c1", "mix2m", "multi_vm", "lvl5", "pae"])
def test_invariants(name):
    assert pins.check_invariants(wl(name)) == []


@pytest.mark.parametrize("name", sorted(SPECS))
def test_generated_batches_are_conflict_free(name):
    from oracle import Oracle
    w = wl(name)
    o = Oracle.from_workload(w)
    assert o.check_conflicts(w.requests, w.epoch_end) is None


def test_conflict_checker_plants():
    """Planted batches: table frames walked in any epoch (read or written, past a
    first fault, PAE root, EPT tables), aliased writes, overlaps in one epoch."""
    assert pins.check_conflict_plants() == []


@pytest.mark.parametrize("name", ["c1", "multi_vm", "lvl5_1g", "prot", "pae_prot"])
def test_results_only_mode_matches_full_batch(name):
    """Results do not depend on bytes or A/D: the results-only walk equals the full batch."""
    import numpy as np
    from oracle import Oracle
    w = wl(name)
    full = Oracle.from_workload(w).batch(w.requests)
    o = Oracle.from_workload(w)
    a0 = [a.copy() for a in o.arenas]
    p0 = o.pool.copy()
    only = o.batch_results(w.requests)
    assert np.array_equal(full[0], only[0]) and np.array_equal(full[1], only[1])
    assert all(np.array_equal(a, b) for a, b in zip(a0, o.arenas)) and np.array_equal(p0, o.pool)


@pytest.mark.parametrize("name", ["c1", "multi_vm", "lvl5_1g", "prot", "pae_prot", "epochs", "ept_faults"])
def test_ad_only_mode_matches_full_batch(name):
    """The A/D-only walk gives the full batch's results, fault list and
    page-table frames, and moves no payload byte."""
    import numpy as np
    from oracle import Oracle
    w = wl(name)
    full = Oracle.from_workload(w)
    fr = full.batch(w.requests)
    o = Oracle.from_workload(w)
    a0 = [a.copy() for a in o.arenas]
    p0 = o.pool.copy()
    ad = o.batch_ad(w.requests)
    assert np.array_equal(fr[0], ad[0]) and np.array_equal(fr[1], ad[1])
    assert np.array_equal(p0, o.pool)
    for v in w.vms:
        pages = pins.table_pages(w, v.vm)
        got = o.arenas[v.vm].reshape(-1, 4096)
        exp = full.arenas[v.vm].reshape(-1, 4096)
        assert np.array_equal(got[pages], exp[pages]), f"vm {v.vm}: table frames differ"
        rest = np.ones(len(got), bool)
        rest[pages] = False
        assert np.array_equal(got[rest], a0[v.vm].reshape(-1, 4096)[rest]), f"vm {v.vm}: payload bytes moved"
    assert any(not np.array_equal(a, b) for a, b in zip(a0, o.arenas)), "no A/D bit was set"


@pytest.mark.parametrize("name", ["multi_vm", "epochs", "lvl5", "prot", "pae", "ept_faults"])
@pytest.mark.parametrize("threads", [3, 8])
def test_threaded_batch_equals_sequential(name, threads):
    """Each epoch's requests split over threads (the CPU baseline's N-thread
    leg) give the sequential batch's results, faults, arenas and pool."""
    import numpy as np
    from oracle import Oracle
    w = wl(name)
    seq = Oracle.from_workload(w)
    sr, sf = seq.batch(w.requests)
    par = Oracle.from_workload(w)
    pr, pf = par.batch_mt(w.requests, w.epoch_end, threads=threads)
    assert np.array_equal(sr, pr) and np.array_equal(sf, pf)
    assert all(np.array_equal(a, b) for a, b in zip(seq.arenas, par.arenas))
    assert np.array_equal(seq.pool, par.pool)
    ad = Oracle.from_workload(w)
    ar, af = ad.batch_mt(w.requests, w.epoch_end, threads=threads, ad_only=True)
    assert np.array_equal(sr, ar) and np.array_equal(sf, af)
    with pytest.raises(ValueError):
        ad.batch_mt(w.requests, w.epoch_end[:-1] if len(w.epoch_end) > 1 else [1], threads=threads)


@pytest.mark.parametrize("per", [1, 2])
def test_vm_chunked_replay_equals_full(per):
    """With a pool range per VM, the requests of a chunk of VMs replayed alone
    (other arenas absent, other pool ranges zero) give that chunk's arenas and
    pool ranges exactly as the whole batch does: the full-size GPU checks
    replay big workloads this way."""
    import numpy as np
    from oracle import Oracle
    from test_gpu_fullsize import _pool_ranges, _sub_epochs, _vm_chunks
    w = wl("multi_vm")
    assert w.pool_vm is not None and len(w.vms) == 3
    full = Oracle.from_workload(w)
    fr, _ = full.batch(w.requests)
    vm_of = np.array([p.vm for p in w.procs], np.int64)[w.requests["asid"]]
    chunks = _vm_chunks(w, per)
    assert sorted(sum(chunks, [])) == list(range(3))
    for vms in chunks:
        arenas = [w.arena_image(v) if v in vms else np.zeros(4096, np.uint8) for v in range(len(w.vms))]
        pool = np.zeros(w.pool_bytes, np.uint8)
        for lo, ln in _pool_ranges(w, vms):
            gen.fill_bytes(pool[lo:lo + ln], w.seed, gen.POOL_KEY, lo)
        oc = Oracle(arenas, [v.slots for v in w.vms], [(p.vm, p.cr3, p.levels) for p in w.procs], pool)
        idx = np.nonzero(np.isin(vm_of, vms))[0]
        cr, _ = oc.batch_mt(w.requests[idx], _sub_epochs(w, idx), threads=3)
        assert np.array_equal(cr, fr[idx])
        for v in vms:
            assert np.array_equal(oc.arenas[v], full.arenas[v])
        for lo, ln in _pool_ranges(w, vms):
            assert np.array_equal(oc.pool[lo:lo + ln], full.pool[lo:lo + ln])


def test_reuse_pool_ranges_per_vm():
    """Reuse mode: every request's host bytes lie in its VM's pool range, the
    ranges tile the pool, and later epochs reuse bytes of earlier ones."""
    import numpy as np
    for name in ("multi_vm", "lvl5", "epochs"):
        w = wl(name)
        r = w.requests
        vm_of = np.array([p.vm for p in w.procs], np.int64)[r["asid"]]
        lo = w.pool_vm[vm_of, 0]
        hi = lo + w.pool_vm[vm_of, 1]
        assert np.all((r["host"] >= lo) & (r["host"] + r["len"].astype(np.uint64) <= hi))
        assert np.array_equal(w.pool_vm[1:, 0], np.cumsum(w.pool_vm[:, 1])[:-1])
        assert int(w.pool_vm[:, 1].sum()) == w.pool_bytes
        if len(w.epoch_end) > 1:
            e1 = int(w.epoch_end[0])
            assert np.any(r["host"][e1:] < np.max(r["host"][:e1] + r["len"][:e1]))


# ------------------------------------------------------------------ EPT --
@pytest.mark.parametrize("name", ["ept", "ept_1g", "c1", "multi_vm", "lvl5", "pae"])
def test_ept_equals_memslots(name):
    """An EPT that maps every slot as the memslots do changes nothing."""
    sp = SPECS[name] if SPECS[name].ept else SPECS[name].replace(ept=True)
    assert pins.check_ept_equivalence(gen.make_workload(sp)) == []


@pytest.mark.parametrize("name", ["ept_faults", "ept_lvl5", "ept_pae"])
def test_ept_faults_follow_the_leaves(name):
    assert pins.check_ept_faults(wl(name)) == []


def test_ept_root_checked():
    import numpy as np
    from oracle import Oracle
    w = wl("ept")
    v = w.vms[0]
    for bad in (v.ept_root + 8, v.arena_bytes, v.arena_bytes - 2048):
        with pytest.raises(ValueError):
            Oracle([np.zeros(v.arena_bytes, np.uint8)], [v.slots], [(0, w.procs[0].cr3, 4)], w.pool_image(),
                   ept=[bad])


@pytest.mark.parametrize("name", ["ept", "pae", "lvl5"])
def test_ept_map_equals_memslots(name):
    """Mapping pages through an EPT that mirrors the memslots changes nothing."""
    sp = SPECS[name] if SPECS[name].ept else SPECS[name].replace(ept=True)
    assert pins.check_ept_map_equivalence(gen.make_workload(sp)) == []


@pytest.mark.parametrize("name", ["ept_faults", "ept_pae"])
def test_ept_map_bad_pool_frame(name):
    assert pins.check_ept_map_bad_pool(wl(name)) == []
