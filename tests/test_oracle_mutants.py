"""The pins catch plausible mistakes.

Each case copies the oracle source, plants one mistake (a dropped term, a
wrong bit, a swapped operand, an off-by-one), builds it on the CPU and runs
the pin checks against it: at least one pin must fail.  The real oracle is
never modified.
"""
import os
import subprocess

import pytest

import pins
from workload import gen

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "oracle.c")

MUTANTS = {
    "index_mask_8bit": ("uint64_t idx = (gva >> shift) & 511;", "uint64_t idx = (gva >> shift) & 255;"),
    "index_shift_off_by_one_level": ("uint32_t shift = 12 + 9 * (uint32_t)(lvl - 1);",
                                     "uint32_t shift = 12 + 9 * (uint32_t)(lvl - 1) + (lvl == 2);"),
    "user_bit_not_accumulated": ("user_ok &= (int)((e >> 2) & 1);", "user_ok &= 1;"),
    "write_bit_not_accumulated": ("write_ok &= (int)((e >> 1) & 1);", "write_ok &= (int)((e >> 1) & 1) | (lvl > 1);"),
    "dirty_on_reads": ("if (write && i + 1 == w->npath) want |= (uint8_t)ORC_D;",
                       "if (i + 1 == w->npath) want |= (uint8_t)ORC_D;"),
    "accessed_only_on_leaf": ("uint8_t want = (uint8_t)ORC_A;",
                              "uint8_t want = (i + 1 == w->npath) ? (uint8_t)ORC_A : 0;"),
    "pat_bit_reserved": ("uint64_t rsvd = (size - 1) & ~((1ull << 13) - 1);",
                         "uint64_t rsvd = (size - 1) & ~((1ull << 12) - 1);"),
    "large_frame_keeps_low_bits": ("frame = e & ORC_ADDR_MASK & ~(size - 1);", "frame = e & ORC_ADDR_MASK;"),
    "ps_at_level4_allowed": ("if (lvl >= 4 && (e & ORC_PS)) {", "if (lvl >= 5 && (e & ORC_PS)) {"),
    "user_write_order_swapped": ("    if (!user_ok) {\n        w->code = ORC_PROT_USER;",
                                 "    if (!user_ok && !(write && !write_ok)) {\n        w->code = ORC_PROT_USER;"),
    "fault_gva_page_base": ("res->fault_gva = lo;", "res->fault_gva = page;"),
    "bytes_done_counts_fault_page": ("res->bytes_done = lo - req->gva;", "res->bytes_done = hi - req->gva;"),
    "slot_end_inclusive": ("if (gpa >= sl->gpa && gpa - sl->gpa < sl->bytes) {",
                           "if (gpa >= sl->gpa && gpa - sl->gpa <= sl->bytes) {"),
    "slot_offset_dropped": ("*hpa = sl->arena_off + (gpa - sl->gpa);", "*hpa = sl->arena_off + gpa;"),
    "canonical_limit_48": ("levels == 3 ? (1ull << 32) : (1ull << 47);", "levels == 3 ? (1ull << 32) : (1ull << 48);"),
    # PAE (the paper's 32-bit platform)
    "pae_root_page_aligned": ("uint64_t pdpt = p->cr3 & 0xFFFFFFE0ull;", "uint64_t pdpt = p->cr3 & 0xFFFFF000ull;"),
    "pae_root_index_bits": ("8 * ((gva >> 30) & 3)", "8 * ((gva >> 29) & 3)"),
    "pae_root_reserved_unchecked": ("if (e & ORC_PAE_PDPTE_RSVD) {", "if (0) {"),
    "pae_high_bits_ignored": ("if (pae && (e & ORC_PAE_RSVD)) {", "if (0) {"),
    "pae_root_gets_accessed": ("        table = e & ORC_ADDR_MASK;\n        top = 2;",
                               "        w->path[w->npath++] = thpa + 8 * ((gva >> 30) & 3);\n"
                               "        table = e & ORC_ADDR_MASK;\n        top = 2;"),
    "pae_root_user_bit": ("        table = e & ORC_ADDR_MASK;\n        top = 2;",
                          "        user_ok &= (int)((e >> 2) & 1);\n        table = e & ORC_ADDR_MASK;\n        top = 2;"),
    "pae_limit_47": ("levels == 3 ? (1ull << 32)", "levels == 3 ? (1ull << 47)"),
    # mapping pages (the guest-table writer)
    "map_link_without_user": ("(root_pae ? ORC_P : (ORC_P | ORC_RW | ORC_US))", "(root_pae ? ORC_P : (ORC_P | ORC_RW))"),
    "map_leaf_always_writable": ("((m->flags & 1) ? ORC_RW : 0)", "ORC_RW"),
    "map_tables_bottom_up": ("return ((uint64_t)(8 - level) << 56)", "return ((uint64_t)level << 56)"),
    "map_earlier_wins": ("    for (uint64_t i = 0; i < n; i++) {\n        if (res[i].code != ORC_OK) continue;\n"
                         "        const orc_map *m = &maps[i];",
                         "    for (uint64_t j = n; j-- > 0;) {\n        uint64_t i = j;\n"
                         "        if (res[i].code != ORC_OK) continue;\n        const orc_map *m = &maps[i];"),
    "map_short_pool_unreported": ("                res[i].code = ORC_NO_POOL;", "                res[i].code = ORC_OK;"),
    "map_new_table_not_zeroed": ("    for (uint64_t k = 0; k < nt; k++) memset(v->arena + pool_hpa[k], 0, 4096);\n", ""),
    "map_pae_root_full_bits": ("(root_pae ? ORC_P :", "(root_pae ? (ORC_P | ORC_RW | ORC_US) :"),
    "map_large_leaf_ignored": ("if (rsvd || (!(pae && lvl == 3) && (e & ORC_PS))) {", "if (rsvd) {"),
    # the EPT walk (a second walk for the guest-physical space)
    "ept_index_mask_8bit": ("uint64_t eoff = table + 8 * ((gpa >> eshift) & 511);",
                            "uint64_t eoff = table + 8 * ((gpa >> eshift) & 255);"),
    "ept_write_without_read_ok": ("if ((e & 3) == 2) return ORC_EPT_MISCONFIG;", "if (0) return ORC_EPT_MISCONFIG;"),
    "ept_table_bits_unchecked": ("if (e & 0xF8) return ORC_EPT_MISCONFIG;", "if (0) return ORC_EPT_MISCONFIG;"),
    "ept_memtype_unchecked": ("if (mt == 2 || mt == 3 || mt == 7)", "if (mt == 7)"),
    "ept_large_leaf_bits_unchecked": ("if (e & (size - 1) & ~0xFFFull) return ORC_EPT_MISCONFIG;",
                                      "if (0) return ORC_EPT_MISCONFIG;"),
    "ept_write_not_anded": ("can_w &= (int)((e >> 1) & 1);", "can_w = (int)((e >> 1) & 1);"),
    "ept_gpa_limit_dropped": ("if (gpa >> 48) return ORC_EPT_VIOLATION;", "if (0) return ORC_EPT_VIOLATION;"),
    "ept_tables_need_read_only": ("uint32_t c = gpa_to_hpa_rec(v, table, ORC_NEED_TABLE, &thpa, rec);",
                                  "uint32_t c = gpa_to_hpa_rec(v, table, ORC_NEED_R, &thpa, rec);"),
    "map_ept_page_table_read_only": ("gpa_to_hpa(v, table, ORC_NEED_TABLE, &thpa);   /* the page table itself */",
                                     "gpa_to_hpa(v, table, ORC_NEED_R, &thpa);   /* the page table itself */"),
    "map_ept_pool_frames_read_only": ("gpa_to_hpa(v, pool[k], ORC_NEED_TABLE, &pool_hpa[k])",
                                      "gpa_to_hpa(v, pool[k], ORC_NEED_R, &pool_hpa[k])"),
    "ept_data_always_read": ("gpa_to_hpa_rec(v, w->gpa, write ? ORC_NEED_W : ORC_NEED_R, &w->hpa, rec)",
                             "gpa_to_hpa_rec(v, w->gpa, ORC_NEED_R, &w->hpa, rec)"),
    "ept_large_leaf_offset_dropped": ("uint64_t h = (e & ORC_ADDR_MASK) | (gpa & (size - 1));",
                                      "uint64_t h = (e & ORC_ADDR_MASK) | (gpa & 0xFFFull);"),
    # the conflict checker (the batch precondition)
    "checker_table_frames_dropped": ("walk_rec(s, p, lo, to_guest, &w, &rd);", "walk_rec(s, p, lo, to_guest, &w, NULL);"),
    "checker_read_vs_write_dropped": ("if (v[i].write && v[i].lo < r_hi && r_req != v[i].req) {", "if (0) {"),
    "checker_table_rule_writes_only": ("        gi[ng++] = d;", "        if (to_guest) gi[ng++] = d;"),
    "checker_table_rule_per_epoch": ("        start = stop;\n        if (n_epochs == 0) break;",
                                     "        start = stop;\n        nt = 0;\n        if (n_epochs == 0) break;"),
    "checker_stops_at_first_fault": ("{ faulted = 1; done = lo - r->gva; continue; }",
                                     "{ faulted = 1; done = lo - r->gva; break; }"),
    "checker_self_alias_allowed": ("        if (v[i].lo < w_hi) {", "        if (v[i].lo < w_hi && w_req != v[i].req) {"),
    "checker_pae_root_unrecorded": ("        note_read(rec, roff);\n", ""),
    "checker_ept_reads_unrecorded": ("        note_read(rec, eoff);\n        uint64_t e = load64(v->arena + eoff);\n        if ((e & 7) == 0)",
                                     "        uint64_t e = load64(v->arena + eoff);\n        if ((e & 7) == 0)"),
    "copy_direction_swapped": ("        if (to_guest)\n            memcpy(g, h, hi - lo);",
                               "        if (!to_guest)\n            memcpy(g, h, hi - lo);"),
    "ad_before_fault_check": ("        if (w.code != ORC_OK) {\n            res->bytes_done",
                              "        if (w.npath) set_ad(s, p, &w, to_guest);\n"
                              "        if (w.code != ORC_OK) {\n            res->bytes_done"),
    "cr3_low_bits_used": ("uint64_t table = p->cr3 & ORC_ADDR_MASK;", "uint64_t table = p->cr3 & ~0x7ull;"),
    "copy_whole_page": ("            memcpy(h, g, hi - lo);", "            memcpy(h, g, hi - lo + (hi - lo < 4096));"),
    # the per-process FIFO translation cache
    "fifo_is_lru": ("    if (slot >= 0 && (!write || f->writable[slot])) {\n        f->hits++;\n        return 1;",
                    "    if (slot >= 0 && (!write || f->writable[slot])) {\n        f->hits++;\n"
                    "        uint64_t v = f->vpn[slot];\n        uint8_t wr = f->writable[slot];\n"
                    "        for (uint32_t k = (slot + cap - f->head) % cap; k + 1 < f->n; k++) {\n"
                    "            f->vpn[(f->head + k) % cap] = f->vpn[(f->head + k + 1) % cap];\n"
                    "            f->writable[(f->head + k) % cap] = f->writable[(f->head + k + 1) % cap];\n        }\n"
                    "        f->vpn[(f->head + f->n - 1) % cap] = v;\n        f->writable[(f->head + f->n - 1) % cap] = wr;\n"
                    "        return 1;"),
    "fifo_nine_entries": ("    const uint32_t cap = s->fifo_entries;", "    const uint32_t cap = s->fifo_entries - 1;"),
    "fifo_inserts_failed_walks": ("    f->misses++;\n    if (!ok) return 0;", "    f->misses++;"),
    "fifo_ignores_write_rights": ("if (slot >= 0 && (!write || f->writable[slot])) {", "if (slot >= 0) {"),
    "fifo_looks_past_fault": ("        if (s->fifo) fifo_lookup(s, req->asid, lo >> 12, to_guest, w.code == ORC_OK);\n",
                              "        if (s->fifo) fifo_lookup(s, req->asid, lo >> 12, to_guest, w.code == ORC_OK);\n"
                              "        if (s->fifo && w.code != ORC_OK && hi < end) fifo_lookup(s, req->asid, hi >> 12, 0, 0);\n"),
    # mapping pages in the EPT (the other half of the mapping routine)
    "ept_map_link_rw_only": ("parent, l + 1, gpa), pool[k] | ORC_EPT_RWX);", "parent, l + 1, gpa), pool[k] | 3ull);"),
    "ept_map_leaf_no_memtype": ("m->hpa | (m->flags & 7u) | ORC_EPT_WB);", "m->hpa | (m->flags & 7u));"),
    "ept_map_earlier_wins": ("    /* 4. leaves, in index order */\n    for (uint64_t i = 0; i < n; i++) {\n"
                             "        if (res[i].code != ORC_OK) continue;\n        const orc_ept_map *m",
                             "    /* 4. leaves, in index order */\n    for (uint64_t i = n; i-- > 0;) {\n"
                             "        if (res[i].code != ORC_OK) continue;\n        const orc_ept_map *m"),
    "ept_map_large_leaf_split": ("        if (lvl <= 3 && (e & 0x80)) return ORC_RESERVED;      /* a large leaf on the path */\n",
                                 "        if (lvl <= 3 && (e & 0x80)) { *missing = lvl; return ORC_OK; }\n"),
    "ept_map_write_only_ok": ("perms == 0 || (perms & 3u) == 2u) {", "perms == 0) {"),
    "ept_map_short_pool_unreported": ("    if (nt > n_pool) {   /* 2. not enough pool pages: nothing is written */",
                                      "    if (nt > n_pool + 1) {   /* 2. not enough pool pages: nothing is written */"),
}

_SMALL = {}


def _small(name):
    if name not in _SMALL:
        _SMALL[name] = gen.make_workload(pins.small_specs()[name])
    return _SMALL[name]


def _build(tmp_path, name):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-O1", "-std=gnu11", "-fPIC", "-shared", "-pthread", str(path), "-o", str(lib)])
    return str(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, name):
    lib = _build(tmp_path, name)
    checks = [
        lambda: pins.check_golden(lib),
        lambda: pins.check_identity(lib),
        lambda: pins.check_roundtrip(_small("mix2m"), lib, per_proc=3000),
        lambda: pins.check_roundtrip(_small("lvl5_1g"), lib, per_proc=3000),
        lambda: pins.check_bruteforce(_small("prot"), lib, max_requests=60),
        lambda: pins.check_ad_closed_form(_small("c1"), lib),
        lambda: pins.check_roundtrip(_small("pae"), lib, per_proc=3000),
        lambda: pins.check_ad_closed_form(_small("pae"), lib),
        lambda: pins.check_golden_maps(lib),
        lambda: pins.check_map_properties(_small("mix2m"), lib),
        lambda: pins.check_map_properties(_small("pae"), lib),
        lambda: pins.check_ept_equivalence(_small("ept"), lib),
        lambda: pins.check_ept_faults(_small("ept_faults"), lib),
        lambda: pins.check_ept_map_bad_pool(_small("ept_faults"), lib),
        lambda: pins.check_conflict_plants(lib),
        lambda: pins.check_golden_fifo(lib),
        lambda: pins.check_golden_ept_maps(lib),
        lambda: pins.check_ept_map_properties(_small("ept_faults"), lib),
    ]
    for c in checks:
        if c():
            return
    pytest.fail(f"no pin caught mutant {name}")
