"""Walker counts and step limits up to the library's maxima (1024 each), in
every form and walk schedule, against the CPU oracle element by element:
rounds of 64 walkers, walks longer than a wavefront (a deletion's winner is
then replayed by one lane), and single-walker, single-step updates."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2505_02741_amd import workloads as W

from gpu_helpers import compare_batch, compare_state, make_pair

pytestmark = pytest.mark.gpu

BATCHED = 4  # DYG_FLAG_BATCHED


@pytest.mark.parametrize("flags,tune", [(0, None), (BATCHED, None), (BATCHED, (8, 1, 4, 0)),
                                        (BATCHED, (8, 1, 0, 0))],
                         ids=["plain", "head-tail", "range", "queue"])
def test_walker_and_step_limits(flags, tune):
    from paper_2505_02741_amd import dygrass as D

    wl = W.make_workload("mesh128", side=8, ins=24, dels=24, batches=2)
    rng = np.random.default_rng(31)
    for b in wl.batches:
        b.s = rng.choice([1, 63, 64, 65, 300, D.MAX_WALKERS], b.size).astype(np.uint16)
        b.L = rng.choice([1, 64, 65, 400, D.MAX_STEPS], b.size).astype(np.uint16)
    o, d = make_pair(wl, flags=flags)
    try:
        if tune:
            D.dyg_set_tuning(d.ctx, *tune)
        for t, b in enumerate(wl.batches):
            compare_batch(o, d, b, tag=f"limits {flags} {tune} batch {t}")
        compare_state(o, d, f"limits {flags} {tune}")
        st = d.stats()
        assert st["walk_steps"] == o.steps_total
        assert st["walk_alg_bytes"] == o.alg_bytes_total
    finally:
        d.close()
        o.close()
