"""Weights whose quantised values reach 2^29 and beyond (up to the 2^32 - 1
clamp): the walks then sum a row's candidate weights in 64 bits.  Both ways
in: heavy from the initial graph (a small reference weight), and heavy edges
inserted into a light graph (later batches walk across them)."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2505_02741_amd import workloads as W

from gpu_helpers import compare_batch, compare_state, make_pair, run_parity, say

pytestmark = pytest.mark.gpu

BATCHED = 4  # DYG_FLAG_BATCHED


@pytest.mark.parametrize("flags", [0, BATCHED])
def test_heavy_from_the_start(flags):
    # weights U[0.5,2) against w_ref = 0.005: quantised 100x to 400x 2^24,
    # clamped at 2^32 - 1 from 256x on
    wl = W.make_workload("mesh128", side=10, ins=120, dels=80, batches=3)
    run_parity(wl, tag=f"heavy init flags={flags}", w_ref=0.005, flags=flags)


@pytest.mark.parametrize("flags", [0, BATCHED])
def test_heavy_edges_inserted_later(flags):
    wl = W.make_workload("grid64", side=30, ins=150, batches=4)
    rng = np.random.default_rng(12)
    es = W.EdgeSet(wl.G)
    # a first batch of local insertions with weights up to 10^4 x the largest
    # initial weight, then the workload's own batches over the changed graph
    p, q = W.local_insertions_lattice(es, 30, 2, 200, rng, np.zeros(0, np.int64))
    z = np.zeros(0, np.uint32)
    heavy = W.Batch(p.astype(np.uint32), q.astype(np.uint32),
                    rng.choice([5.0, 500.0, 5e4], p.size), z, z)
    es.apply(es.key(heavy.iu, heavy.iv), np.zeros(0, np.int64))
    later = []
    for t in range(3):
        pp, qq = W.local_insertions_lattice(es, 30, 2, 150, rng, np.zeros(0, np.int64))
        du, dv = W.uniform_deletions(es, 60, rng)
        b = W.Batch(pp.astype(np.uint32), qq.astype(np.uint32), rng.uniform(1, 10, pp.size),
                    du.astype(np.uint32), dv.astype(np.uint32))
        es.apply(es.key(b.iu, b.iv), es.key(b.du, b.dv))
        later.append(b)
    o, d = make_pair(wl, flags=flags)
    try:
        compare_batch(o, d, heavy, tag="heavy insertions")
        compare_state(o, d, "after heavy insertions")
        for t, b in enumerate(later):
            say(f"  after heavy, batch {t}")
            compare_batch(o, d, b, tag=f"after heavy {t}")
            compare_state(o, d, f"after heavy {t}")
    finally:
        d.close()
        o.close()
