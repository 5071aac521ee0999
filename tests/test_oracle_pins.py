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
