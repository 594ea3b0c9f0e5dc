"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a temporary copy of the C oracle (on the CPU,
never on a GPU), builds it, and runs the pin suites (walk rules, and the
deletion repair) against the broken build: they must fail.  The real oracle
is untouched.
"""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dyg_oracle.c")

MUTANTS = {
    # the previous vertex still counts towards the total weight
    "backtrack_total": ("if ((long)row->e[i].nbr != prev) tot += row->e[i].qw;",
                        "tot += row->e[i].qw;"),
    # off-by-one in the cumulative-weight search
    "select_ge": ("if (run > target) {", "if (run >= target) {"),
    # hit tested before the distortion threshold
    "hit_before_K": ("    if (has_K && w_pq * R > K) break; /* distortion threshold exceeded */\n"
                     "    if (x == q) {\n      hit = 1;\n      break;\n    }",
                     "    if (x == q) {\n      hit = 1;\n      break;\n    }\n"
                     "    if (has_K && w_pq * R > K) break;"),
    # threshold on >= instead of >
    "K_ge": ("if (has_K && w_pq * R > K) break;", "if (has_K && w_pq * R >= K) break;"),
    # wrong word in the Philox round
    "philox_word": ("    uint32_t n1 = lo1;", "    uint32_t n1 = hi1;"),
    # transposed output words
    "word_order": ("uint32_t lo = x[2 * (t & 1u)], hi = x[2 * (t & 1u) + 1];",
                   "uint32_t lo = x[2 * (t & 1u) + 1], hi = x[2 * (t & 1u)];"),
    # conductance summed instead of resistance
    "R_adds_w": ("    R = R + r;", "    R = R + 1.0 / r;"),
    # ties of the minimum resolved to the last walker
    "winner_last": ("if (win == 0xFFFF || res[k].R < rmin) {",
                    "if (win == 0xFFFF || res[k].R <= rmin) {"),
    # decision inverted
    "accept_inverted": ("fl = (uint8_t)!anyh;", "fl = (uint8_t)anyh;"),
    # deleted sparsifier edges stay in H
    "keep_deleted_in_H": ("    if (inH[j]) og_remove(&o->H, du[j], dv[j]);", ""),
    # truncation instead of round-half-even
    "quantize_floor": ("double y = nearbyint(", "double y = floor("),
    # bounce allowed although the policy is TERMINATE
    "always_bounce": ("if (bounce && prev >= 0) forced_back = 1;",
                      "if (prev >= 0) forced_back = 1;"),
    # --- deletion repair (Sec. III-C) ---
    # the first hitting walker wins whatever its resistance
    "winner_first_hit": ("if (win == 0xFFFF || res[k].R < rmin) {", "if (win == 0xFFFF) {"),
    # a hit whose sum overflowed names no walker
    "winner_skips_inf": ("if (win == 0xFFFF || res[k].R < rmin) {", "if (res[k].R < rmin) {"),
    # another hitting walker's path is recovered (the last one that hit)
    "recover_last_hitter": ("const uint32_t *path = traj + (size_t)win * (Li + 1);\n"
                            "        uint32_t plen = res[win].steps + 1;",
                            "uint32_t lw = win;\n"
                            "        for (uint32_t k = 0; k < si; ++k) if (res[k].hit) lw = k;\n"
                            "        const uint32_t *path = traj + (size_t)lw * (Li + 1);\n"
                            "        uint32_t plen = res[lw].steps + 1;"),
    # path edges already in H are recovered again
    "recover_keeps_H_edges": ("          if (og_has(&o->H, a, b)) continue;\n"
                              "          int seen = 0;",
                              "          int seen = 0;"),
    # an edge the path repeats is listed twice
    "recover_no_dedup": ("          if (seen) continue;\n", ""),
    # the path is taken from its far end
    "recover_reversed": ("          uint32_t a = path[t], b = path[t + 1];",
                         "          uint32_t a = path[plen - 1 - t], b = path[plen - 2 - t];"),
    # fallback: the least weight (largest resistance) instead of the largest
    "fallback_min_weight": ("if (best < 0 || row->e[t].r < row->e[best].r) best = (long)t;",
                            "if (best < 0 || row->e[t].r > row->e[best].r) best = (long)t;"),
    # fallback: ties go to the larger neighbour id
    "fallback_ties_larger": ("if (best < 0 || row->e[t].r < row->e[best].r) best = (long)t;",
                             "if (best < 0 || row->e[t].r <= row->e[best].r) best = (long)t;"),
    # fallback: edges already in H are candidates too
    "fallback_ignores_H": ("            if (og_has(&o->H, ends[z], row->e[t].nbr)) continue;\n",
                           ""),
    # an inserted weight whose 1/w overflows is accepted
    "weight_inf_resistance": ("static int weight_ok(double w) { return w > 0.0 && !isinf(w) && "
                              "!isinf(1.0 / w); }",
                              "static int weight_ok(double w) { return w > 0.0 && !isinf(w); }"),
}

# --- initial sparsifier (maximum spanning forest + keyed off-tree sample) ---
MUTANTS.update({
    # minimum instead of maximum spanning forest
    "forest_min_weight": ("if (x->w != y->w) return x->w > y->w ? -1 : 1;",
                          "if (x->w != y->w) return x->w < y->w ? -1 : 1;"),
    # weight ties to the larger edge index
    "forest_ties_larger": ("  return x->e < y->e ? -1 : (x->e > y->e ? 1 : 0);\n}\n\ntypedef struct {\n"
                           "  uint64_t key;",
                           "  return x->e > y->e ? -1 : (x->e < y->e ? 1 : 0);\n}\n\ntypedef struct {\n"
                           "  uint64_t key;"),
    # an edge closing a cycle is kept
    "forest_keeps_cycles": ("    if (a == b) continue;\n    parent[a] = b;",
                            "    parent[a] = b;"),
    # the sample takes the largest keys
    "sample_largest": ("const o_kedge *x = (const o_kedge *)a, *y = (const o_kedge *)b;\n"
                       "  if (x->key != y->key) return x->key < y->key ? -1 : 1;",
                       "const o_kedge *x = (const o_kedge *)a, *y = (const o_kedge *)b;\n"
                       "  if (x->key != y->key) return x->key > y->key ? -1 : 1;"),
    # off by one in the sample: the smallest key is skipped
    "sample_skips_first": ("for (uint64_t i = 0; i < n_off && i < n_extra; ++i) {",
                           "for (uint64_t i = 1; i < n_off && i <= n_extra; ++i) {"),
})

# --- variants of the update rule ---
MUTANTS.update({
    # loop erasure switched off
    "le_noop": ("if (o->variant & ORC_VAR_LOOP_ERASED) {", "if (0) {"),
    # the cut drops the vertex met again
    "le_cut_short": ("if (z < len) len = z + 1;", "if (z < len) len = z;"),
    # the even walkers are the ones that start at the second endpoint
    "both_ends_parity": ("const int flip = (o->variant & ORC_VAR_BOTH_ENDS) && (k & 1u);",
                         "const int flip = (o->variant & ORC_VAR_BOTH_ENDS) && !(k & 1u);"),
    # the two-stage order never repairs H before the insertion walks
    "two_stage_noop": ("if (two) o_add_recovered(o, n_del, rofs, rec_a, rec_b, nrec);",
                       "if (0) o_add_recovered(o, n_del, rofs, rec_a, rec_b, nrec);"),
})

PIN_FILES = ("test_oracle_pins.py", "test_oracle_recovery.py", "test_oracle_sparsifier.py",
             "test_oracle_variants.py")


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not unique"
    mutated = tmp_path / "mut.c"
    mutated.write_text(text.replace(old, new))
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC",
                    "-shared", "-o", str(lib), str(mutated), "-lm"], check=True)
    env = dict(os.environ, DYG_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *(os.path.join(ROOT, "tests", f) for f in PIN_FILES)],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins accept mutant {name}:\n{r.stdout[-2000:]}"
