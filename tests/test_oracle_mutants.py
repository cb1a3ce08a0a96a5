"""Planted mistakes in the oracle (CPU only) must each fail at least one pin.

Each mutant is a one-line textual change of oracle/knng_oracle.c, compiled to
a temporary library and run against tests/test_oracle_pins.py in a child
process. A mutant that passes every pin would show a gap in the pins.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "knng_oracle.c")

MUTANTS = {
    "reverse_neighbours_dropped": ("for (int64_t r = roff[u]; r < roff[u + 1]; ++r) {",
                                   "for (int64_t r = roff[u]; r < roff[u]; ++r) {"),
    "tie_break_reversed": ("return da < db || (da == db && ia < ib);",
                           "return da < db || (da == db && ia > ib);"),
    "no_new_to_old_flip": ("if (f == ORC_NEW) {", "if (0) {"),
    "distance_drops_last_dim": ("for (int64_t j = 0; j < d; ++j) {", "for (int64_t j = 0; j + 1 < d; ++j) {"),
    "old_keeps_new_members": ("if (!in_new) old_raw[co++] = old_raw[i];", "old_raw[co++] = old_raw[i];"),
    "duplicate_tuples_kept": ("if (i > 0 && cmp_cand(&pool[i - 1], &pool[i]) == 0) continue;", ";"),
    "new_new_pairs_skipped": ("for (int32_t j = i + 1; j < nnew[u]; ++j) {", "for (int32_t j = i + 1; j < 0; ++j) {"),
    "hash_constant_typo": ("0x94D049BB133111EBULL", "0x94D049BB133111EAULL"),
    "init_allows_self": ("if ((int64_t)c >= u) c += 1;", ";"),
    "merge_readds_listed_ids": ("if (!in_list) all[n++] = cand[i];", "all[n++] = cand[i];"),
    "weight_not_symmetric": ("uint32_t a = (uint32_t)(u < x ? u : x), b = (uint32_t)(u < x ? x : u);",
                             "uint32_t a = (uint32_t)x, b = (uint32_t)u;"),
    "greedy_scans_list_of_spot_index": ("const int32_t *nb = ids + (int64_t)prev * K;",
                                        "const int32_t *nb = ids + (spot - 1) * K;"),
    "greedy_inverse_not_written": ("sigma_inv[spot] = node;", ";"),
    "greedy_takes_placed_nodes": ("if (!placed[nb[k]]) node = nb[k];", "node = nb[k];"),
    "new_new_proposes_one_way": ("prop[o++] = (orc_prop){nw[j], nw[i], D};",
                                 "prop[o++] = (orc_prop){nw[i], nw[j], D};"),
    "new_old_proposes_one_way": ("prop[o++] = (orc_prop){od[j], nw[i], D};",
                                 "prop[o++] = (orc_prop){nw[i], od[j], D};"),
    "cap_floor": ("double r = ceil(rho * (double)K);", "double r = floor(rho * (double)K);"),
    "hash_ab_swapped": ("return orc_mix64(st ^ (((uint64_t)a << 32) | (uint64_t)b));",
                        "return orc_mix64(st ^ (((uint64_t)b << 32) | (uint64_t)a));"),
    "hash_t_dropped": ("uint64_t st = orc_mix64(s ^ t);", "uint64_t st = orc_mix64(s);"),
    "merge_keeps_repeated_candidates": ("if (i > 0 && cand[i].id == cand[i - 1].id) continue;", ";"),
    "entered_ids_flagged_old": ("if (f == 2) { f = ORC_NEW; ++c; }", "if (f == 2) { f = ORC_OLD; ++c; }"),
    "turbo_counts_whole_pool": ("nf[pool[i].flag == ORC_NEW ? 0 : 1] += 1;", "{ nf[0] += 1; nf[1] += 1; }"),
    "turbo_coin_skipped": ("if (mode == ORC_TURBO &&", "if (0 &&"),
    "block_takes_all_later_owners": ("const int64_t lo = N * (int64_t)b / B, hi = N * (int64_t)(b + 1) / B;",
                                     "const int64_t lo = N * (int64_t)b / B, hi = N;"),
    "block_flips_dropped": ("memcpy(flags + u * K, f2 + u * K, (size_t)K);", ";"),
    "block_outside_owners_join": ("nnew[u] = 0;", ";"),
    "turbo_coin_uses_k": ("* nf[pool[i].flag == ORC_NEW ? 0 : 1] >= ((uint64_t)C << 32))",
                          "* nf[pool[i].flag == ORC_NEW ? 0 : 1] >= ((uint64_t)K << 32))"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation anchor not found: " + old
    with tempfile.TemporaryDirectory() as tmp:
        c = os.path.join(tmp, "mut.c")
        so = os.path.join(tmp, "libmut.so")
        open(c, "w").write(src.replace(old, new, 1))
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", so, c, "-lm"])
        env = dict(os.environ, KNNG_ORACLE_LIB=so, OMP_NUM_THREADS="4")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                           env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
        assert r.returncode != 0, f"mutant {name} passed every pin:\n{r.stdout[-2000:]}"
