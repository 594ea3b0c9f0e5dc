"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a temporary copy of the C oracle (on the CPU,
never on a GPU), builds it, and runs the pin suite against the broken build:
the suite must fail.  The real oracle is untouched.
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
    "winner_last": ("if (res[k].R < rmin) {", "if (res[k].R <= rmin) {"),
    # decision inverted
    "accept_inverted": ("fl = (uint8_t)!anyh;", "fl = (uint8_t)anyh;"),
    # deleted sparsifier edges stay in H
    "keep_deleted_in_H": ("    if (inH[j]) og_remove(&o->H, du[j], dv[j]);", ""),
    # truncation instead of round-half-even
    "quantize_floor": ("double y = nearbyint(", "double y = floor("),
    # bounce allowed although the policy is TERMINATE
    "always_bounce": ("if (bounce && prev >= 0) forced_back = 1;",
                      "if (prev >= 0) forced_back = 1;"),
}


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
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins accept mutant {name}:\n{r.stdout[-2000:]}"
