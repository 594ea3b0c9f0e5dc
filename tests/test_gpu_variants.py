"""Variants of the update rule in the library, against the oracle's same
variant element by element: walkers from both endpoints, loop-erased
recovery, the two-stage batch (deletions and their recoveries before the
insertion walks), their combination, and unweighted selection (a reference
weight so large that every quantised weight is 1)."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2505_02741_amd import workloads as W

from gpu_helpers import make_pair, run_parity, say

pytestmark = pytest.mark.gpu

BATCHED = 4
BOTH, LOOP, TWO = 1, 2, 4


def _mesh():
    return W.make_workload("mesh128", side=12, ins=150, dels=150, batches=5)


def _rmat():
    return W.make_workload("rmat22", scale=12, batches=4, size_lo=50, size_hi=1500)


@pytest.mark.parametrize("variant", [BOTH, LOOP, BOTH | LOOP], ids=["both", "loop", "both+loop"])
@pytest.mark.parametrize("flags", [0, BATCHED], ids=["plain", "batched"])
def test_variant_parity(variant, flags):
    run_parity(_mesh(), tag=f"mesh variant {variant}", flags=flags, variant=variant)
    run_parity(_rmat(), tag=f"rmat variant {variant}", flags=flags, variant=variant)


def test_loop_erased_long_walks_one_lane_replay():
    """Step limits above 64: the winner is replayed by one lane, which erases
    loops as it goes."""
    wl = W.make_workload("mesh128", side=8, ins=60, dels=80, batches=3)
    run_parity(wl, tag="loop L=120", L=120, variant=LOOP)
    run_parity(wl, tag="both+loop L=120 batched", L=120, variant=BOTH | LOOP, flags=BATCHED)


@pytest.mark.parametrize("variant", [TWO, TWO | BOTH | LOOP], ids=["two", "all"])
def test_two_stage_parity(variant):
    run_parity(_mesh(), tag=f"mesh two-stage {variant}", variant=variant)
    run_parity(_rmat(), tag=f"rmat two-stage {variant}", variant=variant)


def test_two_stage_with_pool_growth():
    """Lean pools: the first stage's phase 4 runs short of H slots and the
    library grows H's pool between the stages."""
    wl = W.make_workload("mesh128", side=10, ins=200, dels=300, batches=3)
    run_parity(wl, tag="two-stage lean", variant=TWO, flags=1)  # DYG_FLAG_LEAN_POOLS


def test_two_stage_refused_where_unsupported():
    from paper_2505_02741_amd import dygrass as D

    wl = W.make_workload("grid64", batches=1)
    with pytest.raises(D.DygError):
        make_pair(wl, variant=TWO, flags=BATCHED)
    o, d = make_pair(wl, variant=TWO)
    try:
        with D.DygServer() as srv, pytest.raises(D.DygError):
            srv.add_graph(d)
    finally:
        d.close()
        o.close()


def test_unweighted_selection_parity():
    """A reference weight of 1e300 quantises every weight to 1: the choice is
    uniform over the candidates (the paper's "randomly chosen neighbour")."""
    run_parity(_mesh(), tag="uniform selection", w_ref=1e300)
    run_parity(_rmat(), tag="uniform selection batched", w_ref=1e300, flags=BATCHED)
