"""Checks that pin the CPU oracle to facts other than itself.

Each ``check_*`` function returns a list of failure strings (empty = pass) and
takes an optional ``lib_path`` so the mutation test can run the same checks
against deliberately broken builds of the oracle and show they fail.

Pins used (none re-types the oracle's own code):
  * hand-derived x86-64 walks, A/D updates and copies (tests/golden);
  * encode -> decode: the generator encodes tables from an explicit leaf map
    and the oracle's walk must reproduce that map for every leaf, and report
    unmapped addresses at the level where the encoded path ends;
  * per-byte brute force: every byte of a request translated on its own must
    give the chunked copy's bytes, bytes_done and fault;
  * a textbook special case: identity tables with one memslot at arena
    offset 0 make every successful copy equal to plain memcpy;
  * invariants: round trips, untouched bytes outside requests, A/D equal to
    a closed form computed from the encoded map without walking.
"""
from __future__ import annotations

import json
import os

import numpy as np

from oracle import CODES, Oracle
from oracle.oracle import SLOT_DTYPE, XLAT_SET_AD, XLAT_WRITE
from workload import REQ_DTYPE, gen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "walk_x86_64.json")
H = lambda s: int(s, 16)  # noqa: E731


# ----------------------------------------------------------------- golden --
def golden_worlds():
    with open(GOLDEN) as f:
        return json.load(f)["worlds"]


def build_golden(world, lib_path=None, pool_bytes=0x4000):
    arena = np.zeros(H(world["arena_bytes"]), np.uint8)
    gen.fill_bytes(arena, 77, 3)
    for t in world["table_frames_arena_off"]:
        arena[H(t):H(t) + 4096] = 0
    for e in world["entries"]:
        arena[H(e["arena_off"]):H(e["arena_off"]) + 8] = np.frombuffer(
            H(e["value"]).to_bytes(8, "little"), np.uint8)
    slots = np.zeros(len(world["slots"]), SLOT_DTYPE)
    for i, s in enumerate(world["slots"]):
        slots[i] = (H(s["gpa"]), H(s["bytes"]), H(s["arena_off"]))
    pool = np.zeros(pool_bytes, np.uint8)
    gen.fill_bytes(pool, 78, 4)
    ept = [H(world["ept_root"])] if "ept_root" in world else None
    o = Oracle([arena], [slots], [(0, H(world["cr3"]), world["levels"])], pool, lib_path=lib_path, ept=ept)
    return o, arena, pool


def _u64(arena, off):
    return int.from_bytes(arena[off:off + 8].tobytes(), "little")


def check_golden(lib_path=None):
    fails = []
    for w in golden_worlds():
        o, arena, pool = build_golden(w, lib_path)
        for q in w["queries"]:
            x = o.translate(0, [H(q["gva"])], XLAT_WRITE if q["write"] else 0)[0]
            got = (int(x["code"]), int(x["level"]), int(x["gpa"]), int(x["hpa"]), int(x["page_shift"]))
            exp = (q["code"], q["level"], H(q["gpa"]), H(q["hpa"]), q["shift"])
            if got != exp:
                fails.append(f"{w['name']} walk {q['gva']} w={q['write']}: got {got} expected {exp} ({q['why']})")
        # an invalid process id
        x = o.translate(5, [0x1000])[0]
        if int(x["code"]) != CODES["INVALID"]:
            fails.append(f"{w['name']} invalid asid gave code {int(x['code'])}")
        if "ad_after_set_ad_write" in w:
            ad = w["ad_after_set_ad_write"]
            o, arena, pool = build_golden(w, lib_path)
            o.translate(0, [H(ad["gva"])], XLAT_WRITE | XLAT_SET_AD)
            for e in ad["expect"]:
                if _u64(arena, H(e["arena_off"])) != H(e["value"]):
                    fails.append(f"{w['name']} A/D at {e['arena_off']}: {hex(_u64(arena, H(e['arena_off'])))}"
                                 f" expected {e['value']}")
        for c in w.get("copies", []):
            o, arena, pool = build_golden(w, lib_path)
            a0, p0 = arena.copy(), pool.copy()
            req = np.zeros(1, REQ_DTYPE)
            req[0] = (H(c["gva"]), 0, H(c["len"]), 0, c["dir"], (0, 0, 0), 0)
            r = o.copy(req[0])
            got = (int(r["code"]), int(r["level"]), int(r["bytes_done"]), int(r["fault_gva"]))
            exp = (c["code"], c["level"], H(c["bytes_done"]), H(c["fault_gva"]))
            if got != exp:
                fails.append(f"{w['name']} copy {c['gva']}+{c['len']} dir {c['dir']}: got {got} expected {exp}")
            a_exp, p_exp = a0.copy(), p0.copy()
            for pc in c["pieces"]:
                ao, po, n = H(pc["arena_off"]), H(pc["pool_off"]), H(pc["len"])
                if c["dir"] == 0:
                    p_exp[po:po + n] = a0[ao:ao + n]
                else:
                    a_exp[ao:ao + n] = p0[po:po + n]
            for e in c["ad"]:
                a_exp[H(e["arena_off"]):H(e["arena_off"]) + 8] = np.frombuffer(
                    H(e["value"]).to_bytes(8, "little"), np.uint8)
            if not np.array_equal(arena, a_exp):
                bad = np.nonzero(arena != a_exp)[0]
                fails.append(f"{w['name']} copy {c['gva']} dir {c['dir']}: {len(bad)} arena bytes differ, first {hex(bad[0])}")
            if not np.array_equal(pool, p_exp):
                bad = np.nonzero(pool != p_exp)[0]
                fails.append(f"{w['name']} copy {c['gva']} dir {c['dir']}: {len(bad)} pool bytes differ, first {hex(bad[0])}")
    return fails


def check_golden_maps(lib_path=None):
    """The hand-derived map batches: per-map results, frames used, every entry
    written, new tables zeroed, and no other arena byte changed."""
    from oracle.oracle import MAP_DTYPE
    fails = []
    for w in golden_worlds():
        if "maps" not in w:
            continue
        gm = w["maps"]
        o, arena, pool = build_golden(w, lib_path)
        a0 = arena.copy()
        m = np.zeros(len(gm["batch"]), MAP_DTYPE)
        for i, b in enumerate(gm["batch"]):
            m[i] = (H(b["gva"]), H(b["gpa"]), b["flags"], 0)
        res, used = o.map_pages(0, m, [H(x) for x in gm["pool"]])
        if used != gm["used"]:
            fails.append(f"{w['name']} maps: {used} pool frames used, expected {gm['used']}")
        for i, b in enumerate(gm["batch"]):
            got = (int(res[i]["code"]), int(res[i]["level"]), int(res[i]["bytes_done"]))
            exp = (b["code"], b["level"], 4096 if b["code"] == 0 else 0)
            if got != exp:
                fails.append(f"{w['name']} map {b['gva']}: got {got} expected {exp} ({b['why']})")
        a_exp = a0.copy()
        for z in gm["zeroed"]:
            a_exp[H(z):H(z) + 4096] = 0
        for e in gm["expect"]:
            a_exp[H(e["arena_off"]):H(e["arena_off"]) + 8] = np.frombuffer(H(e["value"]).to_bytes(8, "little"), np.uint8)
        if not np.array_equal(arena, a_exp):
            bad = np.nonzero(arena != a_exp)[0]
            fails.append(f"{w['name']} maps: {len(bad)} arena bytes differ, first {hex(int(bad[0]))}")
    return fails


def free_frames(wl, vm, count, rng):
    """Guest frames no table and no data page of the encoded map uses."""
    v = wl.vms[vm]
    used = set(int(x) for x in v.pt_gfn)
    for p in wl.procs:
        if p.vm != vm:
            continue
        for lv, fr in zip(p.leaf_level, p.leaf_frame):
            n = 1 << (9 * (int(lv) - 1))
            base = int(fr) >> 12
            used.update(range(base, base + n)) if n <= 512 else used.update((base, base + n - 1))
    nfr = v.mem_bytes >> 12
    cand = np.setdiff1d(np.arange(nfr, dtype=np.int64), np.fromiter(used, np.int64))
    return (rng.choice(cand, count, replace=False).astype(np.uint64) << np.uint64(12))


def usable_frames(wl, vm, frames):
    """The frames a VM's EPT maps readable and writable (by the generator's
    leaf list); all of them for a memslot VM."""
    lf = wl.vms[vm].ept_leaf
    if lf is None:
        return frames
    from workload.gen import EPT_LEAF_OK
    kind = lf["kind"][np.searchsorted(lf["gpa"], frames, side="right") - 1]
    return frames[kind == EPT_LEAF_OK]


def map_batch(wl, rng, n=600):
    """Maps for process 0: remaps of mapped 4 KiB pages, pages in mapped and in
    empty regions, pages inside large leaves, out-of-range pages, duplicates."""
    from oracle.oracle import MAP_DTYPE
    p = wl.procs[0]
    lim = {3: 1 << 32, 4: 1 << 47, 5: 1 << 56}[p.levels]
    lvl = p.leaf_level
    g = []
    k = n // 6
    g += list(p.leaf_va[lvl == 1][rng.integers(0, max(1, int((lvl == 1).sum())), k)])        # remaps
    big = np.nonzero(lvl >= 2)[0]
    if len(big):                                                                            # inside large leaves
        j = big[rng.integers(0, len(big), k)]
        g += list(p.leaf_va[j] + (rng.integers(0, 512, k).astype(np.uint64) << np.uint64(12)))
    vb = p.vmas[rng.integers(0, len(p.vmas), k)]                                            # around the VMAs
    g += list(vb[:, 0] + vb[:, 1] + (rng.integers(0, 4096, k).astype(np.uint64) << np.uint64(12)))
    g += list((rng.integers(1, lim >> 12, k, dtype=np.uint64) << np.uint64(12)))            # anywhere
    g += [np.uint64(lim), np.uint64(lim + 4096)]                                            # out of range
    g = np.array(g, np.uint64)
    g = np.concatenate([g, g[rng.integers(0, len(g), k)]])                                  # duplicates
    rng.shuffle(g)
    m = np.zeros(len(g), MAP_DTYPE)
    m["gva"] = g
    m["gpa"] = rng.integers(0, wl.vms[p.vm].mem_bytes >> 12, len(g)).astype(np.uint64) << np.uint64(12)
    m["flags"] = rng.integers(0, 2, len(g))
    return m


def expected_new_tables(wl, m):
    """Tables the maps need and the encoded map lacks, counted from the
    generator's table sets (no walk), and the expected per-map codes."""
    p = wl.procs[0]
    lim = {3: 1 << 32, 4: 1 << 47, 5: 1 << 56}[p.levels]
    tabs = _leaf_lookup(p)
    li = find_leaf(p, tabs, m["gva"])
    code = np.zeros(len(m), np.int64)
    code[m["gva"] >= np.uint64(lim)] = CODES["NONCANONICAL"]
    inside_large = (li >= 0) & (p.leaf_level[np.maximum(li, 0)] >= 2) & (code == 0)
    code[inside_large] = CODES["RESERVED"]
    new = set()
    for gva in m["gva"][code == 0]:
        for L in range(1, p.levels):
            ids = p.tables[L][0]
            t = int(gva) >> (12 + 9 * L)
            pos = np.searchsorted(ids, np.uint64(t))
            if not (pos < len(ids) and int(ids[pos]) == t):
                new.add((L, t))
    return code, len(new)


def check_map_properties(wl, lib_path=None, seed=3):
    """Map a batch with the oracle, then check it against the encoded map.
    Needs a world whose encoded tables are all reachable (p_upper_np = 0)."""
    assert wl.spec.p_upper_np == 0
    fails = []
    rng = np.random.default_rng(seed)
    p = wl.procs[0]
    m = map_batch(wl, rng)
    code, n_new = expected_new_tables(wl, m)
    pool = free_frames(wl, p.vm, n_new + 5, rng)
    # too small a pool: nothing is written
    o = Oracle.from_workload(wl, lib_path=lib_path)
    a0 = [a.copy() for a in o.arenas]
    if n_new:
        res, used = o.map_pages(0, m, pool[:n_new - 1])
        if used != 0 or not all(np.array_equal(a, b) for a, b in zip(a0, o.arenas)):
            fails.append("short pool: something was written")
        if np.any(res["code"][code == 0] != CODES["NO_POOL"]):
            fails.append("short pool: a map did not report NO_POOL")
    res, used = o.map_pages(0, m, pool)
    if not np.array_equal(res["code"].astype(np.int64), code):
        i = int(np.nonzero(res["code"].astype(np.int64) != code)[0][0])
        fails.append(f"map {hex(int(m['gva'][i]))}: code {int(res['code'][i])} expected {int(code[i])}")
    if used != n_new:
        fails.append(f"{used} new tables, the encoded map lacks {n_new}")
    ok = np.nonzero(code == 0)[0]
    last = {}
    for i in ok:
        last[int(m["gva"][i])] = i
    idx = np.array(sorted(last.values()), np.int64)
    x = o.translate(0, m["gva"][idx])
    if np.any(x["code"] != 0) or np.any(x["gpa"] != m["gpa"][idx]) or np.any(x["page_shift"] != 12):
        fails.append("a mapped page does not translate to its (last) frame")
    wrote = o.translate(0, m["gva"][idx], XLAT_WRITE)
    if np.any((wrote["code"] == CODES["PROT_WRITE"]) != (m["flags"][idx] & 1 == 0)):
        fails.append("R/W of a mapped page does not follow its flags")
    # pages the batch left alone translate as before
    mapped = set(last)
    keep = np.array([i for i in range(len(p.leaf_va)) if p.leaf_present[i] and p.leaf_level[i] == 1
                     and int(p.leaf_va[i]) not in mapped][:3000], np.int64)
    if len(keep):
        before = Oracle.from_workload(wl, lib_path=lib_path).translate(0, p.leaf_va[keep])
        after = o.translate(0, p.leaf_va[keep])
        if not np.array_equal(before, after):
            fails.append("a page outside the batch changed its translation")
    return fails


# ------------------------------------------------------- encode -> decode --
def _leaf_lookup(p):
    """Map page-granular keys to leaf indices using the encoder's own map."""
    tabs = {}
    for L in (1, 2, 3):
        m = np.nonzero(p.leaf_level == L)[0]
        keys = p.leaf_va[m] >> np.uint64(12 + 9 * (L - 1))
        order = np.argsort(keys)
        tabs[L] = (keys[order], m[order])
    return tabs


def find_leaf(p, tabs, va):
    """Index of the leaf covering each va, -1 if none (from the encoded map)."""
    va = np.asarray(va, np.uint64)
    out = np.full(len(va), -1, np.int64)
    for L in (1, 2, 3):
        keys, idx = tabs[L]
        if len(keys) == 0:
            continue
        k = va >> np.uint64(12 + 9 * (L - 1))
        pos = np.minimum(np.searchsorted(keys, k), len(keys) - 1)
        hit = keys[pos] == k
        out = np.where(hit & (out < 0), idx[pos], out)
    return out


def expected_unmapped_level(p, va):
    """Level of the deepest encoded table on the path of an unmapped address."""
    va = np.asarray(va, np.uint64)
    lvl = np.full(len(va), p.levels, np.int64)
    for L in range(p.levels - 1, 0, -1):
        ids = p.tables[L][0]
        k = va >> np.uint64(12 + 9 * L)
        pos = np.minimum(np.searchsorted(ids, k), max(len(ids) - 1, 0))
        has = (ids[pos] == k) if len(ids) else np.zeros(len(va), bool)
        lvl = np.where(has, L, lvl)
    return lvl


def check_roundtrip(wl, lib_path=None, per_proc=20000, seed=5):
    fails = []
    o = Oracle.from_workload(wl, lib_path=lib_path)
    rng = np.random.default_rng(seed)
    for p in wl.procs:
        n = len(p.leaf_va)
        sel = rng.choice(n, min(n, per_proc), replace=False) if n > per_proc else np.arange(n)
        size = np.uint64(1) << (np.uint64(12) + np.uint64(9) * (p.leaf_level[sel].astype(np.uint64) - np.uint64(1)))
        off = (rng.integers(0, 2**62, len(sel), dtype=np.uint64) % size)
        va = p.leaf_va[sel] + off
        x = o.translate(p.asid, va)
        pres = p.leaf_present[sel]
        exp_gpa = p.leaf_frame[sel] + off
        ok_codes = x["code"][pres]
        if np.any(ok_codes != 0):
            i = np.nonzero(ok_codes != 0)[0][0]
            fails.append(f"asid {p.asid}: mapped va {hex(int(va[pres][i]))} gave code {int(ok_codes[i])}")
            continue
        if np.any(x["gpa"][pres] != exp_gpa[pres]):
            i = np.nonzero(x["gpa"][pres] != exp_gpa[pres])[0][0]
            fails.append(f"asid {p.asid}: va {hex(int(va[pres][i]))} gpa {hex(int(x['gpa'][pres][i]))} "
                         f"expected {hex(int(exp_gpa[pres][i]))}")
            continue
        exp_hpa = gen.gpa_to_arena(wl.vms[p.vm].slots, exp_gpa[pres])
        if np.any(x["hpa"][pres].astype(np.int64) != exp_hpa):
            fails.append(f"asid {p.asid}: hpa differs from the memslot layout")
        if np.any(x["page_shift"][pres] != (12 + 9 * (p.leaf_level[sel][pres].astype(np.int64) - 1))):
            fails.append(f"asid {p.asid}: page_shift differs from the encoded leaf size")
        npres = ~pres
        if np.any(x["code"][npres] != CODES["NOT_PRESENT"]) or \
                np.any(x["level"][npres] != p.leaf_level[sel][npres]):
            fails.append(f"asid {p.asid}: not-present leaves not reported at their own level")
        # unmapped addresses: random user addresses that no leaf covers
        lim = 1 << {3: 32, 4: 47, 5: 56}[p.levels]
        cand = rng.integers(0, lim, 4000, dtype=np.uint64)
        # plus addresses just past each VMA (share upper tables with mapped ones)
        cand = np.concatenate([cand, p.vmas[:, 0] + p.vmas[:, 1], p.vmas[:, 0] - np.uint64(4096)])
        cand = cand[find_leaf(p, _leaf_lookup(p), cand) < 0]
        xu = o.translate(p.asid, cand)
        if np.any(xu["code"] != CODES["NOT_PRESENT"]):
            fails.append(f"asid {p.asid}: an unmapped address did not fault NOT_PRESENT")
        elif np.any(xu["level"].astype(np.int64) != expected_unmapped_level(p, cand)):
            fails.append(f"asid {p.asid}: unmapped address fault level differs from the encoded path")
    return fails


# ---------------------------------------------------------- brute force --
def check_bruteforce(wl, lib_path=None, max_requests=None):
    """Per-byte translation vs the chunked copy, on a fresh oracle state."""
    fails = []
    o = Oracle.from_workload(wl, lib_path=lib_path)
    a0 = [a.copy() for a in o.arenas]
    p0 = o.pool.copy()
    reqs = wl.requests if max_requests is None else wl.requests[:max_requests]
    res, _ = o.batch(reqs)
    # expected, request by request in order on a second state
    o2 = Oracle([a.copy() for a in a0], [v.slots for v in wl.vms],
                [(p.vm, p.cr3, p.levels) for p in wl.procs], p0.copy(), lib_path=lib_path)
    for i, r in enumerate(reqs):
        n = int(r["len"])
        gva = int(r["gva"])
        to_guest = int(r["dir"]) == 1
        if n == 0:
            continue
        b = np.arange(n, dtype=np.uint64) + np.uint64(gva)
        x = o2.translate(int(r["asid"]), b, XLAT_WRITE if to_guest else 0)
        bad = np.nonzero(x["code"] != 0)[0]
        done = int(bad[0]) if len(bad) else n
        exp = (done, gva + done if len(bad) else 0, int(x["code"][done]) if len(bad) else 0,
               int(x["level"][done]) if len(bad) else 0)
        got = (int(res[i]["bytes_done"]), int(res[i]["fault_gva"]), int(res[i]["code"]), int(res[i]["level"]))
        if got != exp:
            fails.append(f"request {i}: chunked {got} vs per-byte {exp}")
            continue
        ar = o2.arenas[wl.procs[int(r["asid"])].vm]
        hp = x["hpa"][:done].astype(np.int64)
        host = int(r["host"])
        if to_guest:
            ar[hp] = o2.pool[host:host + done]
        else:
            o2.pool[host:host + done] = ar[hp]
        # A/D: set through a walk of the first copied byte of every copied page
        if done:
            pg = np.unique(b[:done] >> np.uint64(12))
            firsts = np.maximum(pg << np.uint64(12), np.uint64(gva))
            o2.translate(int(r["asid"]), firsts, (XLAT_WRITE if to_guest else 0) | XLAT_SET_AD)
    for v in range(len(wl.vms)):
        if not np.array_equal(o.arenas[v], o2.arenas[v]):
            fails.append(f"vm {v}: arena bytes differ between chunked and per-byte application")
    if not np.array_equal(o.pool, o2.pool):
        fails.append("pool bytes differ between chunked and per-byte application")
    return fails


# ------------------------------------------------------- identity tables --
def identity_world(n_pages=96, levels=4, seed=9):
    """Identity-mapped user pages [base, base + n_pages*4K) with one memslot at
    arena offset 0, built by a tiny recursive encoder independent of the
    generator (tables allocated top-down from the end of guest memory).
    levels 3 is PAE: the root is a 4-entry table of P-only entries at byte
    0x40 of its frame, indexed by address bits 31:30."""
    rng = np.random.default_rng(seed)
    base = 0x40_0000  # 4 MiB
    mem = 16 << 20
    arena = np.zeros(mem, np.uint8)
    gen.fill_bytes(arena, seed, 1)
    next_frame = [mem - 4096]
    tables = {}

    def alloc():
        f = next_frame[0]
        next_frame[0] -= 4096
        arena[f:f + 4096] = 0
        return f

    root = alloc()
    if levels == 3:
        root += 0x40  # the PAE root table is 32-byte aligned, not page aligned

    def put(table, idx, val):
        arena[table + 8 * idx: table + 8 * idx + 8] = np.frombuffer(int(val).to_bytes(8, "little"), np.uint8)

    def get(table, idx):
        return int.from_bytes(arena[table + 8 * idx: table + 8 * idx + 8].tobytes(), "little")

    present = rng.random(n_pages) > 0.1
    for k in range(n_pages):
        va = base + 4096 * k
        table = root
        for lvl in range(levels, 1, -1):
            idx = (va >> (12 + 9 * (lvl - 1))) & 511
            if levels == 3 and lvl == 3:
                idx = (va >> 30) & 3
            e = get(table, idx)
            if e & 1:
                table = e & 0x000FFFFFFFFFF000
            else:
                t = alloc()
                put(table, idx, t | (0x1 if (levels == 3 and lvl == 3) else 0x7))
                table = t
        put(table, (va >> 12) & 511, (va | 0x7) if present[k] else 0)
    slots = np.zeros(1, SLOT_DTYPE)
    slots[0] = (0, mem, 0)
    return arena, slots, root, base, present


def check_identity(lib_path=None, seed=9):
    fails = []
    for levels in (3, 4, 5):
        arena, slots, root, base, present = identity_world(levels=levels, seed=seed)
        pool = np.zeros(1 << 20, np.uint8)
        gen.fill_bytes(pool, seed, 2)
        o = Oracle([arena], [slots], [(0, root, levels)], pool, lib_path=lib_path)
        rng = np.random.default_rng(seed + levels)
        hostpos = 0
        for _ in range(60):
            gva = base + int(rng.integers(0, 96 * 4096 - 1))
            n = int(rng.integers(1, min(20000, base + 96 * 4096 - gva) + 1))
            d = int(rng.integers(0, 2))
            req = np.zeros(1, REQ_DTYPE)
            req[0] = (gva, hostpos, n, 0, d, (0, 0, 0), 0)
            pre_a, pre_p = arena.copy(), pool.copy()
            r = o.copy(req[0])
            pages = [(gva + i) >> 12 for i in range(0, n)]
            first_bad = next((i for i in range(n) if not present[((gva + i) >> 12) - (base >> 12)]), n)
            if int(r["bytes_done"]) != first_bad:
                fails.append(f"identity L{levels}: bytes_done {int(r['bytes_done'])} expected {first_bad}")
                break
            k = first_bad
            if d == 0:
                exp_p = pre_p.copy()
                exp_p[hostpos:hostpos + k] = pre_a[gva:gva + k]   # memcpy(pool+host, arena+gva, k)
                if not np.array_equal(pool, exp_p):
                    fails.append(f"identity L{levels}: guest->host differs from memcpy")
                    break
            else:
                data = arena[gva:gva + k]
                if not np.array_equal(data, pre_p[hostpos:hostpos + k]):
                    fails.append(f"identity L{levels}: host->guest differs from memcpy")
                    break
            del pages
            hostpos = (hostpos + n + 64) % ((1 << 20) - 20100)
    return fails


# -------------------------------------------------------------- A/D form --
def expected_ad(wl, reqs, res):
    """Final page-table bytes from the encoded map and the copied pages only."""
    exp = {}
    for v in wl.vms:
        exp[v.vm] = v.pt_data.copy()
    pos = {}
    for v in wl.vms:
        order = np.argsort(v.pt_gfn)
        pos[v.vm] = (v.pt_gfn[order], order)
    tabs = {p.asid: _leaf_lookup(p) for p in wl.procs}
    A, D = np.uint64(0x20), np.uint64(0x40)
    for i, r in enumerate(reqs):
        done = int(res[i]["bytes_done"])
        if done == 0:
            continue
        p = wl.procs[int(r["asid"])]
        gva = int(r["gva"])
        pages = np.arange(gva >> 12, ((gva + done - 1) >> 12) + 1, dtype=np.uint64) << np.uint64(12)
        li = find_leaf(p, tabs[p.asid], pages)
        assert np.all(li >= 0)
        gfns, order = pos[p.vm]
        tgt = exp[p.vm]

        def orbits(gfn, idx, bits):
            k = order[np.searchsorted(gfns, gfn)]
            np.bitwise_or.at(tgt, (k, idx.astype(np.int64)), bits)

        lv = p.leaf_level[li]
        orbits(p.leaf_table_gfn[li], p.leaf_index[li], A | (D if int(r["dir"]) == 1 else np.uint64(0)))
        # A on every upper entry of the path; a PAE root entry has no A bit
        for L in range(2, (2 if p.levels == 3 else p.levels) + 1):
            m = lv < L
            if not m.any():
                continue
            ids, tg = p.tables[L]
            va = pages[m]
            t = tg[np.searchsorted(ids, va >> np.uint64(12 + 9 * L))]
            idx = (va >> np.uint64(12 + 9 * (L - 1))) & np.uint64(511)
            orbits(t, idx, A)
    return exp


def check_ad_closed_form(wl, lib_path=None):
    fails = []
    o = Oracle.from_workload(wl, lib_path=lib_path)
    res, _ = o.batch(wl.requests)
    exp = expected_ad(wl, wl.requests, res)
    for v in wl.vms:
        hpa = gen.gpa_to_arena(v.slots, v.pt_gfn << np.uint64(12))
        got = o.arenas[v.vm].reshape(-1, 4096)[(hpa >> 12)].view(np.uint64)
        if not np.array_equal(got, exp[v.vm]):
            nbad = int(np.sum(got != exp[v.vm]))
            fails.append(f"vm {v.vm}: {nbad} page-table entries differ from the A/D closed form")
    return fails


# ------------------------------------------------------------ invariants --
def check_invariants(wl, lib_path=None):
    """Round trips and untouched bytes."""
    fails = []
    o = Oracle.from_workload(wl, lib_path=lib_path)
    a0 = [a.copy() for a in o.arenas]
    p0 = o.pool.copy()
    reqs = wl.requests
    res, faults = o.batch(reqs)
    # fault list: one record per faulting request, ascending
    fidx = np.nonzero(res["code"] != 0)[0]
    if not np.array_equal(faults["req_index"], fidx.astype(np.uint64)):
        fails.append("fault list is not the ascending list of faulting requests")
    # bytes outside requests unchanged: pool changes only inside FROM_GUEST prefixes
    allowed = np.zeros(o.pool.size, bool)
    for i in np.nonzero(reqs["dir"] == 0)[0]:
        h, d = int(reqs[i]["host"]), int(res[i]["bytes_done"])
        allowed[h:h + d] = True
    if np.any((o.pool != p0) & ~allowed):
        fails.append("pool bytes changed outside guest->host request prefixes")
    # arena changes only in page-table frames (A/D) and TO_GUEST prefixes
    for v in wl.vms:
        allowed = np.zeros(o.arenas[v.vm].size, bool)
        hpa = gen.gpa_to_arena(v.slots, v.pt_gfn << np.uint64(12))
        for h in hpa:
            allowed[h:h + 4096] = True
        for i in np.nonzero((reqs["dir"] == 1))[0]:
            p = wl.procs[int(reqs[i]["asid"])]
            if p.vm != v.vm or res[i]["bytes_done"] == 0:
                continue
            g = int(reqs[i]["gva"])
            x = o.translate(int(reqs[i]["asid"]), np.arange(g, g + int(res[i]["bytes_done"]), dtype=np.uint64))
            allowed[x["hpa"].astype(np.int64)] = True
        if np.any((o.arenas[v.vm] != a0[v.vm]) & ~allowed):
            fails.append(f"vm {v.vm}: arena bytes changed outside page tables and host->guest prefixes")
    # round trips, epoch by epoch (requests of one epoch never overlap; across
    # epochs they may reuse guest and pool bytes)
    o2 = Oracle([a.copy() for a in a0], [v.slots for v in wl.vms],
                [(p.vm, p.cr3, p.levels) for p in wl.procs], p0.copy(), lib_path=lib_path)
    pt_mask = []
    for v in range(len(wl.vms)):
        hpa = gen.gpa_to_arena(wl.vms[v].slots, wl.vms[v].pt_gfn << np.uint64(12))
        m = np.zeros(o2.arenas[v].size, bool)
        for h in hpa:
            m[h:h + 4096] = True
        pt_mask.append(m)
    for e0, e1 in wl.epochs():
        ep = reqs[e0:e1]
        # guest -> host -> guest leaves guest data bytes as they were
        fwd = ep.copy()
        fwd["dir"] = 0
        snap = [a.copy() for a in o2.arenas]
        r1, _ = o2.batch(fwd)
        back = fwd.copy()
        back["dir"] = 1
        r2, _ = o2.batch(back)
        if not np.array_equal(r1["bytes_done"], r2["bytes_done"]):
            fails.append(f"epoch [{e0},{e1}) guest->host->guest: bytes_done differ")
        for v in range(len(wl.vms)):
            if np.any((o2.arenas[v] != snap[v]) & ~pt_mask[v]):
                fails.append(f"epoch [{e0},{e1}) guest->host->guest changed guest data bytes in vm {v}")
        # host -> guest -> host brings the pool prefix back
        before = o2.pool.copy()
        r3, _ = o2.batch(back)
        o2.pool[:] = 0
        r4, _ = o2.batch(fwd)
        for i in range(len(ep)):
            h, d = int(ep[i]["host"]), int(r3[i]["bytes_done"])
            if int(r4[i]["bytes_done"]) < d or not np.array_equal(o2.pool[h:h + d], before[h:h + d]):
                fails.append(f"host->guest->host: request {e0 + i} did not come back")
                break
        if fails:
            break
    # every byte of a not-present page faults: requests wholly inside one not-present leaf
    for p in wl.procs[:4]:
        np_idx = np.nonzero(~p.leaf_present)[0][:50]
        for li in np_idx:
            va = int(p.leaf_va[li]) + 5
            q = np.zeros(1, REQ_DTYPE)
            q[0] = (va, 0, 16, p.asid, 0, (0, 0, 0), 0)
            r = o2.copy(q[0])
            if int(r["code"]) != CODES["NOT_PRESENT"] or int(r["bytes_done"]) != 0:
                fails.append(f"asid {p.asid}: read of a not-present page at {hex(va)} did not fault")
                break
    return fails


def check_golden_fifo(lib_path=None):
    """The per-process FIFO translation cache (section 4.2) on a hand-derived
    sequence of copies in the 4-level golden world: cumulative hits and misses
    after every copy, as worked out by hand in the golden file."""
    fails = []
    for w in golden_worlds():
        if "fifo" not in w:
            continue
        o, arena, pool = build_golden(w, lib_path)
        o.fifo_reset(w["fifo"]["entries"])
        for i, st in enumerate(w["fifo"]["steps"]):
            req = np.zeros(1, REQ_DTYPE)
            req[0] = (H(st["gva"]), 0, H(st["len"]), 0, st["dir"], (0, 0, 0), 0)
            o.copy(req[0])
            got = o.fifo_counts(0)
            if got != (st["hits"], st["misses"]):
                fails.append(f"{w['name']} fifo step {i}: (hits, misses) {got}, expected "
                             f"{(st['hits'], st['misses'])} ({st['why']})")
                break
    return fails


def check_fifo_properties(wl, lib_path=None, entries=10):
    """The translation cache changes no result, no arena and no pool byte; its
    lookups per process are exactly the pages the copies translate (up to and
    including each first faulting page); a cache as large as every page a
    process touches misses exactly once per distinct successfully translated
    page plus once per failed walk and per write to a page first held for
    reading."""
    fails = []
    reqs = wl.requests
    base = Oracle.from_workload(wl, lib_path=lib_path)
    br, bf = base.batch(reqs)
    o = Oracle.from_workload(wl, lib_path=lib_path)
    o.fifo_reset(entries)
    r, f = o.batch(reqs)
    if not (np.array_equal(r, br) and np.array_equal(f, bf)):
        fails.append("the cache changed results")
    if not all(np.array_equal(a, b) for a, b in zip(o.arenas, base.arenas)) or not np.array_equal(o.pool, base.pool):
        fails.append("the cache changed memory")
    # lookups = pages translated: every page of a request that copied everything,
    # else the pages up to and including the faulting one
    g = reqs["gva"].astype(np.uint64)
    ln = reqs["len"].astype(np.uint64)
    valid = (r["code"] != CODES["INVALID"]) & (r["code"] != CODES["NONCANONICAL"]) & (ln > 0)
    last = np.where(r["code"] == 0, g + ln - np.uint64(1), r["fault_gva"].astype(np.uint64))
    pages = np.where(valid, (last >> np.uint64(12)) - (g >> np.uint64(12)) + np.uint64(1), np.uint64(0))
    for p in wl.procs:
        m = reqs["asid"] == p.asid
        h, mi = o.fifo_counts(p.asid)
        if h + mi != int(pages[m].sum()):
            fails.append(f"asid {p.asid}: {h + mi} lookups, {int(pages[m].sum())} pages translated")
            break
    # an unbounded cache: misses = first successful translation of each page, each
    # later write to a page held only for reads, and every failed walk
    big = Oracle.from_workload(wl, lib_path=lib_path)
    big.fifo_reset(64)
    sel = np.nonzero(valid & (pages <= 2))[0][:3000]
    held = {}
    exp_miss = {}
    for i in sel:
        q = reqs[i]
        a = int(q["asid"])
        rr = big.copy(q)
        first, npg = int(q["gva"]) >> 12, int(pages[i])
        for k in range(npg):
            vpn = first + k
            ok = not (int(rr["code"]) != 0 and k == npg - 1)
            wr = int(q["dir"]) == 1
            st = held.setdefault(a, {})
            hit = vpn in st and (not wr or st[vpn])
            if not hit:
                exp_miss[a] = exp_miss.get(a, 0) + 1
                if ok:
                    st[vpn] = st.get(vpn, False) or wr
        if sum(len(v) for v in held.values()) > 60 * len(held):
            break
    for a, n in exp_miss.items():
        if len(held[a]) <= 64 and big.fifo_counts(a)[1] != n:
            fails.append(f"asid {a}: a 64-entry cache missed {big.fifo_counts(a)[1]} times, expected {n}")
            break
    return fails


def table_pages(wl, vm):
    """Arena page numbers of every table frame of a VM: its guest page tables
    (through the memslots) and its EPT tables, if it has an EPT."""
    v = wl.vms[vm]
    pages = [(gen.gpa_to_arena(v.slots, v.pt_gfn << np.uint64(12)) >> 12).astype(np.int64)]
    if v.ept_root is not None:
        pages.append((v.ept_off >> np.uint64(12)).astype(np.int64))
    return np.unique(np.concatenate(pages))


def small_specs():
    """Reduced configurations with the named ones' structure, sized for seconds on the CPU."""
    KiB, MiB, GiB = 1 << 10, 1 << 20, 1 << 30
    return {
        "tiny4k": gen.spec("C1", mem_bytes=512 * KiB, n_requests=64, n_slots=2, p_np=0.2, len_hi=12000, seed=11),
        "c1": gen.spec("C1"),
        "mix2m": gen.spec("C2", mem_bytes=64 * MiB, n_requests=400, n_slots=6, len_hi=40000, seed=12),
        "multi_vm": gen.spec("C3", n_vms=3, procs_per_vm=2, mem_bytes=32 * MiB, n_requests=500, len_hi=300000,
                             seed=13),
        "lvl5": gen.spec("C5", n_vms=2, mem_bytes=32 * MiB, mix=(0.6, 0.4, 0.0), n_requests=300, len_hi=100000,
                         seed=14),
        "lvl5_1g": gen.spec("C5", n_vms=1, mem_bytes=3 * GiB // 2, mapped_frac=0.7, mix=(0.02, 0.02, 0.96),
                            n_requests=200, len_hi=100000, seed=15),
        "prot": gen.spec("C2", mem_bytes=16 * MiB, n_requests=300, p_readonly=0.1, p_supervisor=0.05,
                         p_upper_np=0.05, len_hi=20000, seed=16),
        # the paper's 32-bit PAE platform: 4 KiB and 2 MiB pages under a 4-entry root table
        "pae": gen.spec("C2", levels=3, mem_bytes=64 * MiB, n_requests=400, n_slots=6, len_hi=40000, seed=17),
        "pae_prot": gen.spec("C2", levels=3, mem_bytes=16 * MiB, n_requests=300, p_readonly=0.1,
                             p_supervisor=0.05, p_upper_np=0.1, len_hi=20000, seed=18),
        # guest-physical space described by an EPT (a second software walk) instead of memslots
        "ept": gen.spec("C2", mem_bytes=64 * MiB, n_requests=400, n_slots=6, len_hi=40000, seed=21, ept=True),
        "ept_faults": gen.spec("C2", mem_bytes=64 * MiB, n_requests=600, n_slots=6, len_hi=40000, seed=22,
                               ept=True, ept_np=0.03, ept_ro=0.05, ept_mis=0.02),
        "ept_lvl5": gen.spec("C5", n_vms=2, mem_bytes=32 * MiB, mix=(0.6, 0.4, 0.0), n_requests=300,
                             len_hi=100000, seed=23, ept=True, ept_np=0.02, ept_ro=0.04, ept_mis=0.02),
        "ept_pae": gen.spec("C2", levels=3, mem_bytes=64 * MiB, n_requests=400, n_slots=6, len_hi=40000, seed=24,
                            ept=True, ept_np=0.03, ept_ro=0.05, ept_mis=0.02),
        "ept_1g": gen.spec("C5", n_vms=1, mem_bytes=3 * GiB // 2, n_slots=1, mapped_frac=0.7,
                           mix=(0.02, 0.02, 0.96), n_requests=200, len_hi=100000, seed=25, ept=True, ept_align=GiB),
        # long requests (up to 512 pages) over several epochs, for the workgroup walk of large requests
        "large": gen.spec("C3", n_vms=2, procs_per_vm=2, mem_bytes=64 * MiB, n_requests=400, len_hi=2 * MiB,
                          seed=32),
        # many epochs (each fills at most 10% of a VMA) that reuse guest and pool bytes across epochs
        "epochs": gen.spec("C3", n_vms=2, procs_per_vm=2, mem_bytes=32 * MiB, n_requests=3000, len_hi=64 * KiB,
                           rho=0.1, seed=31),
    }


# ------------------------------------------------------------------ EPT --
def check_ept_equivalence(wl, lib_path=None, sample=4000):
    """A world whose EPT maps every slot exactly as its memslots do must give
    the same results, fault list, arena and pool bytes, and translations, in
    EPT mode as in memslot mode."""
    assert wl.spec.ept and wl.spec.ept_np == wl.spec.ept_ro == wl.spec.ept_mis == 0
    fails = []
    e = Oracle.from_workload(wl, lib_path=lib_path)
    m = Oracle([wl.arena_image(v) for v in range(len(wl.vms))], [v.slots for v in wl.vms],
               [(p.vm, p.cr3, p.levels) for p in wl.procs], wl.pool_image(), lib_path=lib_path)
    rng = np.random.default_rng(7)
    for p in wl.procs:
        g = p.leaf_va[rng.integers(0, len(p.leaf_va), min(sample, len(p.leaf_va)))]
        g = g + (rng.integers(0, 4096, len(g)).astype(np.uint64))
        for fl in (0, XLAT_WRITE | XLAT_SET_AD):
            a, b = e.translate(p.asid, g, fl), m.translate(p.asid, g, fl)
            if not np.array_equal(a, b):
                i = int(np.nonzero(a != b)[0][0])
                fails.append(f"asid {p.asid} gva {hex(int(g[i]))} flags {fl}: EPT {a[i]} memslots {b[i]}")
                break
    re_, fe = e.batch(wl.requests)
    rm, fm = m.batch(wl.requests)
    if not np.array_equal(re_, rm) or not np.array_equal(fe, fm):
        fails.append("batch results or fault list differ between EPT and memslot modes")
    for v, (x, y) in enumerate(zip(e.arenas, m.arenas)):
        if not np.array_equal(x, y):
            fails.append(f"vm {v}: arenas differ between EPT and memslot modes")
    if not np.array_equal(e.pool, m.pool):
        fails.append("pools differ between EPT and memslot modes")
    return fails


def check_ept_faults(wl, lib_path=None):
    """With EPT leaves made not present, read-only or misconfigured, every
    data page's outcome follows from the leaf that holds its GPA (taken from
    the generator's list, not from a walk): not present -> EPT_VIOLATION,
    misconfigured -> EPT_MISCONFIG, read-only -> EPT_VIOLATION on writes into
    the guest only; every other page copies."""
    from workload.gen import EPT_LEAF_MIS, EPT_LEAF_NP, EPT_LEAF_RO
    fails = []
    o = Oracle.from_workload(wl, lib_path=lib_path)
    res, _ = o.batch_results(wl.requests)
    kinds = {}
    for v in wl.vms:
        lf = v.ept_leaf
        kinds[v.vm] = lf
    seen = {"viol": 0, "mis": 0, "ok_pages": 0, "table_level": 0}
    for i, (rq, r) in enumerate(zip(wl.requests, res)):
        p = wl.procs[int(rq["asid"])]
        lf = kinds[p.vm]
        wr = int(rq["dir"]) == 1
        end = int(rq["gva"]) + int(rq["len"])
        stop = int(r["fault_gva"]) if r["code"] != 0 else end
        gv = [max(pg, int(rq["gva"])) for pg in range(int(rq["gva"]) & ~0xFFF, stop, 4096)]
        gv = [g for g in gv if g < stop]  # the pages copied before the fault
        if r["code"] != 0 and r["level"] == 0 and r["code"] in (CODES["EPT_VIOLATION"], CODES["EPT_MISCONFIG"]):
            gv.append(int(r["fault_gva"]))
        elif r["code"] in (CODES["EPT_VIOLATION"], CODES["EPT_MISCONFIG"]):
            seen["table_level"] += 1
        if not gv:
            continue
        x = o.translate(p.asid, np.array(gv, np.uint64), XLAT_WRITE if wr else 0)
        for k, g in enumerate(gv):
            gpa = int(x["gpa"][k])
            j = int(np.searchsorted(lf["gpa"], np.uint64(gpa), side="right")) - 1
            if j < 0 or gpa - int(lf["gpa"][j]) >= (1 << int(lf["shift"][j])):
                fails.append(f"request {i}: GPA {hex(gpa)} is in no EPT leaf")
                continue
            kind = int(lf["kind"][j])
            exp = CODES["EPT_VIOLATION"] if kind == EPT_LEAF_NP or (kind == EPT_LEAF_RO and wr) else \
                CODES["EPT_MISCONFIG"] if kind == EPT_LEAF_MIS else 0
            last = k == len(gv) - 1 and r["code"] != 0 and r["level"] == 0
            got = int(r["code"]) if last else 0
            if x["level"][k] != 0 or (x["code"][k] != 0 and x["code"][k] not in (CODES["EPT_VIOLATION"],
                                                                                 CODES["EPT_MISCONFIG"])):
                if last:
                    fails.append(f"request {i}: page {hex(g)} faults above the data page")
                continue
            if got != exp:
                fails.append(f"request {i} page {hex(g)} (GPA {hex(gpa)}, leaf kind {kind}, write {wr}): "
                             f"code {got} expected {exp}")
                break
            seen["viol" if exp == CODES["EPT_VIOLATION"] else "mis" if exp else "ok_pages"] += 1
        if len(fails) > 5:
            break
    if not fails and (seen["viol"] == 0 or seen["mis"] == 0 or seen["ok_pages"] == 0):
        fails.append(f"the world exercises too little: {seen}")
    return fails


def check_ept_map_equivalence(wl, lib_path=None, seed=5):
    """Mapping pages in a VM whose EPT mirrors its memslots gives the same
    results, frames used and arena bytes as in memslot mode, for a short pool
    and for an ample one."""
    assert wl.spec.ept and wl.spec.ept_np == wl.spec.ept_ro == wl.spec.ept_mis == 0
    fails = []
    rng = np.random.default_rng(seed)
    p = wl.procs[0]
    m = map_batch(wl, rng)
    pool = free_frames(wl, p.vm, 3 * len(m), rng)
    e = Oracle.from_workload(wl, lib_path=lib_path)
    s = Oracle([wl.arena_image(v) for v in range(len(wl.vms))], [v.slots for v in wl.vms],
               [(q.vm, q.cr3, q.levels) for q in wl.procs], wl.pool_image(), lib_path=lib_path)
    _, need = Oracle.from_workload(wl, lib_path=lib_path).map_pages(0, m, pool)
    for k in (max(need - 1, 0), len(pool)):
        re_, ue = e.map_pages(0, m, pool[:k])
        rs, us = s.map_pages(0, m, pool[:k])
        if not np.array_equal(re_, rs) or ue != us:
            fails.append(f"pool of {k}: results or frames used differ between EPT and memslot modes")
        if not all(np.array_equal(a, b) for a, b in zip(e.arenas, s.arenas)):
            fails.append(f"pool of {k}: arenas differ between EPT and memslot modes")
    if need == 0:
        fails.append("the batch needs no new table")
    return fails


def check_ept_map_bad_pool(wl, lib_path=None, seed=6):
    """A pool frame the batch takes but the EPT does not map readable and
    writable (not present or read-only, from the generator's leaf list) makes
    the whole batch NO_POOL with nothing written; the same frame placed past
    the frames the batch needs changes nothing."""
    from workload.gen import EPT_LEAF_NP, EPT_LEAF_OK, EPT_LEAF_RO
    fails = []
    rng = np.random.default_rng(seed)
    p = wl.procs[0]
    lf = wl.vms[p.vm].ept_leaf
    m = map_batch(wl, rng)
    cand = free_frames(wl, p.vm, 4000, rng)
    j = np.searchsorted(lf["gpa"], cand, side="right") - 1
    kind = lf["kind"][j]
    good = cand[kind == EPT_LEAF_OK]
    bads = {"not present": cand[kind == EPT_LEAF_NP], "read-only": cand[kind == EPT_LEAF_RO]}
    if len(good) < 2000 or any(len(b) == 0 for b in bads.values()):
        return ["the world has too few free frames of each kind"]
    r0, need = Oracle.from_workload(wl, lib_path=lib_path).map_pages(0, m, good)
    if need < 2:
        return ["the batch needs fewer than two tables"]
    ok = r0["code"] == CODES["OK"]
    for what, bad in bads.items():
        o = Oracle.from_workload(wl, lib_path=lib_path)
        a0 = [a.copy() for a in o.arenas]
        r, used = o.map_pages(0, m, np.concatenate([good[:need // 2], bad[:1], good[need // 2:]]))
        if used != 0 or not all(np.array_equal(a, b) for a, b in zip(a0, o.arenas)):
            fails.append(f"a needed {what} frame: something was written")
        if np.any(r["code"][ok] != CODES["NO_POOL"]) or np.any(r["code"][~ok] != r0["code"][~ok]):
            fails.append(f"a needed {what} frame: maps not reported NO_POOL")
        r2, used2 = Oracle.from_workload(wl, lib_path=lib_path).map_pages(
            0, m, np.concatenate([good[:need], bad[:1]]))
        if used2 != need or not np.array_equal(r2, r0):
            fails.append(f"a {what} frame past the needed ones changed the result")
    return fails


# ------------------------------------------------------ conflict checker --
_ADDR = 0x000FFFFFFFFFF000


def _entry_off(wl, p, i):
    """Arena offset of leaf i's entry (from the encoder's record of where it wrote it)."""
    v = wl.vms[p.vm]
    t = int(gen.gpa_to_arena(v.slots, np.array([int(p.leaf_table_gfn[i]) << 12], np.uint64))[0])
    return t + 8 * int(p.leaf_index[i])


def _set_u64(arena, off, val):
    arena[off:off + 8] = np.frombuffer(int(val).to_bytes(8, "little"), np.uint8)


def _req(gva, host, n, asid, d):
    r = np.zeros(1, REQ_DTYPE)
    r[0] = (gva, host, n, asid, d, (0, 0, 0), 0)
    return r


def _ept_leaf_off(arena, root, gpa):
    """Arena offset of the EPT entry that maps gpa (generator-built EPT; no checks)."""
    table = root
    for lvl in (4, 3, 2, 1):
        off = table + 8 * ((gpa >> (12 + 9 * (lvl - 1))) & 511)
        e = _u64(arena, off)
        if lvl == 1 or (e & 0x80):
            return off, lvl
        table = e & _ADDR


def check_conflict_plants(lib_path=None):
    """The conflict checker against planted batches whose answer follows from
    the batch precondition: a request whose guest bytes lie in a page-table
    frame that some walk loads (same epoch, a later or an earlier epoch, read
    or write, a walk past the walker's first fault, the PAE root table, an EPT
    table), writes to aliased guest pages, and overlaps inside one epoch.
    Each plant rewrites a leaf so that a guest page lands on the frame in
    question; the same requests without the plant must pass."""
    fails = []
    specs = small_specs()
    W, R = gen.TO_GUEST, gen.FROM_GUEST

    def check(tag, o, reqs, ends, want):
        got = o.check_conflicts(np.concatenate(reqs), ends)
        if (got is not None) != want:
            fails.append(f"{tag}: checker says {got}, expected {'a conflict' if want else 'none'}")

    # ---- 4-level world: leaf Y rewritten onto X's leaf table frame
    wl = gen.make_workload(specs["c1"])
    p = wl.procs[0]
    four = np.nonzero((p.leaf_level == 1) & p.leaf_present)[0]
    x = int(four[0])
    fx = int(p.leaf_table_gfn[x]) << 12
    y = int(next(i for i in four if int(p.leaf_table_gfn[i]) << 12 != fx))
    z = int(next(i for i in four if int(p.leaf_table_gfn[i]) != p.leaf_table_gfn[x] and
                 int(p.leaf_table_gfn[i]) != p.leaf_table_gfn[y] and i != y))
    vx, vy, vz = int(p.leaf_va[x]), int(p.leaf_va[y]), int(p.leaf_va[z])

    def world(plant):
        a = wl.arena_image(0)
        if plant:
            off = _entry_off(wl, p, y)
            _set_u64(a, off, (_u64(a, off) & ~_ADDR) | fx)
        return Oracle([a], [wl.vms[0].slots], [(0, p.cr3, p.levels)], wl.pool_image(), lib_path=lib_path)

    yw, yr = _req(vy + 100, 0, 64, 0, W), _req(vy + 100, 0, 64, 0, R)
    xr, zr = _req(vx + 8, 4096, 64, 0, R), _req(vz + 8, 8192, 64, 0, R)
    o0, o1 = world(False), world(True)
    check("unplanted, one epoch", o0, [yw, xr, zr], [3], False)
    check("unplanted, three epochs", o0, [yw, xr, zr], [1, 2, 3], False)
    check("write onto a table walked in the same epoch", o1, [yw, xr], [2], True)
    check("write onto a table walked in a later epoch", o1, [yw, xr], [1, 2], True)
    check("write onto a table walked in an earlier epoch", o1, [xr, yw], [1, 2], True)
    check("read of a table walked in another epoch", o1, [xr, yr], [1, 2], True)
    check("bytes in a table no request walks", o1, [yw, zr], [1, 2], False)

    # ---- a walk past its request's first fault: the walker starts on a page
    # made not present, and its next page's leaf table is the planted one
    nxt = {int(v): i for i, v in zip(four, p.leaf_va[four])}
    starts = [i for i in four if int(p.leaf_index[i]) == 0 and int(p.leaf_va[i]) - 4096 in nxt and
              p.leaf_table_gfn[nxt[int(p.leaf_va[i]) - 4096]] != p.leaf_table_gfn[i]]
    if not starts:
        fails.append("no 2 MiB boundary between two 4 KiB leaf tables in the world")
    else:
        x2 = int(starts[0])
        p0 = nxt[int(p.leaf_va[x2]) - 4096]
        f2 = int(p.leaf_table_gfn[x2]) << 12
        y2 = int(next(i for i in four if p.leaf_table_gfn[i] not in (p.leaf_table_gfn[x2], p.leaf_table_gfn[p0])))
        a = wl.arena_image(0)
        off = _entry_off(wl, p, p0)
        _set_u64(a, off, _u64(a, off) & ~1)          # page before x2: not present
        off = _entry_off(wl, p, y2)
        _set_u64(a, off, (_u64(a, off) & ~_ADDR) | f2)
        o2 = Oracle([a], [wl.vms[0].slots], [(0, p.cr3, p.levels)], wl.pool_image(), lib_path=lib_path)
        walker = _req(int(p.leaf_va[x2]) - 32, 4096, 64, 0, R)   # faults on its first page
        res, _ = o2.batch(walker)
        if int(res[0]["code"]) != CODES["NOT_PRESENT"] or int(res[0]["bytes_done"]) != 0:
            fails.append(f"planted walker should fault at once, got {res[0]}")
        check("write onto a table walked only past a first fault", o2,
              [_req(int(p.leaf_va[y2]) + 8, 0, 64, 0, W), walker], [1, 2], True)

    # ---- aliased writes inside one request: page y+1 rewritten onto y's frame
    nb = [i for i in four if int(p.leaf_va[i]) + 4096 in nxt]
    ya = int(nb[0])
    yb = nxt[int(p.leaf_va[ya]) + 4096]
    a = wl.arena_image(0)
    off = _entry_off(wl, p, yb)
    _set_u64(a, off, (_u64(a, off) & ~_ADDR) | int(p.leaf_frame[ya]))
    o3 = Oracle([a], [wl.vms[0].slots], [(0, p.cr3, p.levels)], wl.pool_image(), lib_path=lib_path)
    span = _req(int(p.leaf_va[ya]) + 100, 0, 4200, 0, W)        # frame bytes 100..203 written twice
    check("one request writing two aliased pages", o3, [span], [1], True)
    check("one request reading two aliased pages", o3, [_req(int(p.leaf_va[ya]) + 100, 0, 4200, 0, R)], [1], False)

    # ---- overlap inside one epoch: a read starting below a write of the same
    # guest bytes (the reader sorts first), and two writers of one pool range
    g = vx + 512
    check("guest read below an overlapping guest write", o0, [_req(g, 0, 64, 0, R), _req(g + 32, 4096, 64, 0, W)],
          [2], True)
    check("the same pair in two epochs", o0, [_req(g, 0, 64, 0, R), _req(g + 32, 4096, 64, 0, W)], [1, 2], False)
    check("two writers of one pool range", o0, [_req(vx + 8, 0, 64, 0, R), _req(vz + 8, 32, 64, 0, R)], [2], True)

    # ---- PAE: a leaf rewritten onto the frame of the 4-entry root table
    wp = gen.make_workload(specs["pae"])
    pp = wp.procs[0]
    fp = np.nonzero((pp.leaf_level == 1) & pp.leaf_present)[0]
    yp, xp = int(fp[0]), int(fp[-1])
    a = wp.arena_image(0)
    off = _entry_off(wp, pp, yp)
    _set_u64(a, off, (_u64(a, off) & ~_ADDR) | (pp.cr3 & ~0xFFF))
    o4 = Oracle([a], [wp.vms[0].slots], [(0, pp.cr3, 3)], wp.pool_image(), lib_path=lib_path)
    check("PAE: write onto the root table's frame", o4,
          [_req(int(pp.leaf_va[yp]) + 2048, 0, 64, 0, W), _req(int(pp.leaf_va[xp]), 4096, 64, 0, R)], [1, 2], True)

    # ---- EPT: the EPT leaf of a guest data page rewritten onto the EPT root table
    we = gen.make_workload(specs["ept"])
    pe, ve = we.procs[0], we.vms[0]
    a = we.arena_image(0)
    fe = np.nonzero((pe.leaf_level == 1) & pe.leaf_present)[0]
    ye = None
    for i in fe:
        eoff, lvl = _ept_leaf_off(a, ve.ept_root, int(pe.leaf_frame[i]))
        if lvl == 1:
            ye = int(i)
            break
    if ye is None:
        fails.append("no guest 4 KiB page with a 4 KiB EPT leaf in the EPT world")
    else:
        xe = int(next(i for i in fe if i != ye))
        reqs = [_req(int(pe.leaf_va[ye]) + 64, 0, 64, 0, W), _req(int(pe.leaf_va[xe]), 4096, 64, 0, R)]
        o5 = Oracle([a.copy()], [ve.slots], [(0, pe.cr3, pe.levels)], we.pool_image(), lib_path=lib_path,
                    ept=[ve.ept_root])
        check("EPT: unplanted", o5, reqs, [1, 2], False)
        _set_u64(a, eoff, (_u64(a, eoff) & ~_ADDR) | ve.ept_root)
        o6 = Oracle([a], [ve.slots], [(0, pe.cr3, pe.levels)], we.pool_image(), lib_path=lib_path,
                    ept=[ve.ept_root])
        check("EPT: write onto the EPT root table", o6, reqs, [1, 2], True)
    return fails


# ------------------------------------------------------------ EPT maps --
def check_golden_ept_maps(lib_path=None):
    """The hand-derived EPT map batch on the EPT golden world: per-map results,
    pool pages used, every entry written, new tables zeroed, no other arena
    byte changed; with the pool one page short, nothing written."""
    from oracle.oracle import EPT_MAP_DTYPE
    fails = []
    for w in golden_worlds():
        if "ept_maps" not in w:
            continue
        gm = w["ept_maps"]
        m = np.zeros(len(gm["batch"]), EPT_MAP_DTYPE)
        for i, b in enumerate(gm["batch"]):
            m[i] = (H(b["gpa"]), H(b["hpa"]), b["flags"], 0)
        o, arena, pool = build_golden(w, lib_path)
        a0 = arena.copy()
        res, used = o.ept_map_pages(0, m, [H(x) for x in gm["pool"]])
        if used != gm["used"]:
            fails.append(f"{w['name']} EPT maps: {used} pool pages used, expected {gm['used']}")
        for i, b in enumerate(gm["batch"]):
            got = (int(res[i]["code"]), int(res[i]["level"]), int(res[i]["bytes_done"]))
            exp = (b["code"], b["level"], 4096 if b["code"] == 0 else 0)
            if got != exp:
                fails.append(f"{w['name']} EPT map {i} {b['gpa']}: got {got} expected {exp} ({b['why']})")
        a_exp = a0.copy()
        for z in gm["zeroed"]:
            a_exp[H(z):H(z) + 4096] = 0
        for e in gm["expect"]:
            a_exp[H(e["arena_off"]):H(e["arena_off"]) + 8] = np.frombuffer(H(e["value"]).to_bytes(8, "little"), np.uint8)
        if not np.array_equal(arena, a_exp):
            bad = np.nonzero(arena != a_exp)[0]
            fails.append(f"{w['name']} EPT maps: {len(bad)} arena bytes differ, first {hex(int(bad[0]))}")
        # one pool page short: every map that would succeed reports NO_POOL, nothing is written
        o, arena, pool = build_golden(w, lib_path)
        a0 = arena.copy()
        res, used = o.ept_map_pages(0, m, [H(x) for x in gm["short_pool"]])
        want = [CODES["NO_POOL"] if b["code"] == 0 else b["code"] for b in gm["batch"]]
        if used != 0 or list(res["code"]) != want or not np.array_equal(arena, a0):
            fails.append(f"{w['name']} EPT maps, short pool: used {used}, codes {list(res['code'])}")
    return fails


def ept_map_batch(wl, vm, n, rng):
    """A mixed EPT map batch for a generated EPT world: GPAs inside the mapped
    guest memory (existing 4 KiB leaves and 2 MiB / 1 GiB regions), GPAs in
    unmapped space far above it (new tables at every level), repeats, and a
    few invalid maps; targets are random arena pages; the pool is arena pages
    no EPT or guest table uses."""
    from oracle.oracle import EPT_MAP_DTYPE
    v = wl.vms[vm]
    pages = v.arena_bytes >> 12
    inside = rng.integers(0, v.mem_bytes >> 12, n).astype(np.uint64) << np.uint64(12)
    far = (np.uint64(1) << np.uint64(40)) + (rng.integers(0, 1 << 20, n).astype(np.uint64) << np.uint64(12))
    gpa = np.where(rng.random(n) < 0.5, inside, far)
    gpa[n // 3: n // 3 + n // 10] = gpa[:n // 10]                        # repeats: the later map wins
    m = np.zeros(n, EPT_MAP_DTYPE)
    m["gpa"] = gpa
    m["hpa"] = rng.integers(0, pages, n).astype(np.uint64) << np.uint64(12)
    m["flags"] = rng.choice(np.array([1, 3, 5, 7], np.uint32), n)
    m["flags"][n - 4] = 2                                                  # write without read
    m["hpa"][n - 3] = np.uint64(v.arena_bytes)                             # outside the arena
    m["gpa"][n - 2] |= np.uint64(8)                                        # unaligned
    m["gpa"][n - 1] = np.uint64(1) << np.uint64(48)                        # past the EPT's reach
    used = set(int(x) >> 12 for x in v.ept_off)
    used.update(int(x) >> 12 for x in gen.gpa_to_arena(v.slots, v.pt_gfn << np.uint64(12)))
    cand = np.setdiff1d(np.arange(pages, dtype=np.int64), np.fromiter(used, np.int64))
    pool = rng.choice(cand, min(len(cand), 4 * n), replace=False).astype(np.uint64) << np.uint64(12)
    return m, pool


def check_ept_map_properties(wl, lib_path=None, n=400, seed=5):
    """On a generated EPT world: each map's outcome and the number of new
    tables follow from the generator's EPT leaf list without a walk; after the
    batch, the oracle's EPT walker takes every mapped GPA to its target page
    with the map's rights and every other sampled GPA where it went before; a
    pool one page short writes nothing."""
    from oracle.oracle import CODES as OC
    fails = []
    rng = np.random.default_rng(seed)
    vm = 0
    v = wl.vms[vm]
    m, pool = ept_map_batch(wl, vm, n, rng)
    from workload.gen import EPT_LEAF_MIS, EPT_LEAF_NP
    lf = v.ept_leaf
    g = lf["gpa"].astype(np.uint64)
    sh = lf["shift"].astype(np.uint64)
    kind = lf["kind"]
    # large leaves that are present (a not-present one is a missing entry);
    # a misconfigured one may be write-without-read (EPT_MISCONFIG) or of a
    # reserved memory type (a large leaf: RESERVED), which the list does not tell
    big1 = {a >> 30: k for a, k in ((int(x), int(k)) for x, s2, k in zip(g, sh, kind)
                                     if s2 == 30 and k != EPT_LEAF_NP)}
    big2 = {a >> 21: k for a, k in ((int(x), int(k)) for x, s2, k in zip(g, sh, kind)
                                     if s2 == 21 and k != EPT_LEAF_NP)}
    pts = set(int(x) >> 21 for x, s2 in zip(g, sh) if s2 == 12)
    pds = set(int(x) >> 30 for x, s2 in zip(g, sh) if s2 <= 21)
    pdpts = set(int(x) >> 39 for x in g)
    need = set()
    allowed = []   # per map: the codes the leaf list allows, and the level
    for i, (a, h, f) in enumerate(zip(m["gpa"], m["hpa"], m["flags"])):
        a, h, f = int(a), int(h), int(f)
        if a & 0xFFF or a >> 48 or h & 0xFFF or h + 4096 > v.arena_bytes or f & ~7 or f == 0 or f & 3 == 2:
            allowed.append(({OC["NONCANONICAL"]}, 0))
        elif a >> 30 in big1:
            mis = big1[a >> 30] == EPT_LEAF_MIS
            allowed.append(({OC["RESERVED"], OC["EPT_MISCONFIG"]} if mis else {OC["RESERVED"]}, 3))
        elif a >> 21 in big2:
            mis = big2[a >> 21] == EPT_LEAF_MIS
            allowed.append(({OC["RESERVED"], OC["EPT_MISCONFIG"]} if mis else {OC["RESERVED"]}, 2))
        else:
            allowed.append(({0}, 0))
            if a >> 39 not in pdpts:
                need.add((3, a >> 39))
            if a >> 30 not in pds:
                need.add((2, a >> 30))
            if a >> 21 not in pts:
                need.add((1, a >> 21))
    exp_code = np.array([0 if c == {0} else -1 for c, _ in allowed])
    o = Oracle.from_workload(wl, lib_path=lib_path)
    sample = np.concatenate([rng.integers(0, v.mem_bytes >> 12, 2000).astype(np.uint64) << np.uint64(12),
                             m["gpa"][exp_code == 0]])
    sample = np.setdiff1d(sample, m["gpa"])
    x0 = [o.ept_xlat(vm, int(a), 0) for a in sample]
    res, used = o.ept_map_pages(vm, m, pool)
    bad = [i for i, (c, lv) in enumerate(allowed) if int(res["code"][i]) not in c or int(res["level"][i]) != lv]
    if bad:
        fails.append(f"EPT maps: {len(bad)} results differ from the leaf list, first map {bad[0]}: "
                     f"{res[bad[0]]} vs codes {allowed[bad[0]]}")
    if used != len(need):
        fails.append(f"EPT maps: {used} new tables, {len(need)} needed by the leaf list")
    last = {}
    for i in range(n):
        if exp_code[i] == 0:
            last[int(m["gpa"][i])] = i
    for a, i in last.items():
        f = int(m["flags"][i])
        for need_bits, ok in ((1, f & 1), (2, f & 2)):
            code, hpa = o.ept_xlat(vm, a, need_bits)
            if ok and (code != 0 or hpa != int(m["hpa"][i])):
                fails.append(f"EPT maps: GPA {a:#x} -> {code}, {hpa:#x}; expected {int(m['hpa'][i]):#x}")
                break
            if not ok and code != OC["EPT_VIOLATION"]:
                fails.append(f"EPT maps: GPA {a:#x} without right {need_bits} gave code {code}")
                break
    x1 = [o.ept_xlat(vm, int(a), 0) for a in sample]
    if x0 != x1:
        k = next(j for j in range(len(x0)) if x0[j] != x1[j])
        fails.append(f"EPT maps: GPA {int(sample[k]):#x} outside the batch moved: {x0[k]} -> {x1[k]}")
    # one pool page short: nothing written
    o2 = Oracle.from_workload(wl, lib_path=lib_path)
    a0 = o2.arenas[vm].copy()
    res2, used2 = o2.ept_map_pages(vm, m, pool[:max(0, len(need) - 1)])
    want = np.where(res["code"] == 0, OC["NO_POOL"], res["code"])
    if len(need) and (used2 != 0 or list(res2["code"]) != list(want) or not np.array_equal(o2.arenas[vm], a0)):
        fails.append("EPT maps: a pool one page short wrote something")
    return fails
