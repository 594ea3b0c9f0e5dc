"""Variants of the update rule in the library, against the oracle's same
variant element by element: walkers from both endpoints, loop-erased
recovery, the two-stage batch (deletions and their recoveries before the
insertion walks), their combination, and unweighted selection (a reference
weight so large that every quantised weight is 1)."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2505_02741_amd import workloads as W

from gpu_helpers import compare_state, make_pair, run_parity, say

pytestmark = pytest.mark.gpu

BATCHED = 4
GRAPH = 8
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


def test_two_stage_batched_form():
    """A batched context (with captured graphs for its other batches) runs a
    two-stage batch with the lockstep walk, launched directly."""
    run_parity(_mesh(), tag="mesh two-stage batched", variant=TWO | BOTH, flags=BATCHED | GRAPH)
    run_parity(_rmat(), tag="rmat two-stage batched", variant=TWO, flags=BATCHED)


def test_two_stage_device_batches():
    """Two-stage batches handed over in device memory, on the library's
    stream and on a caller stream, in both forms."""
    import torch

    from paper_2505_02741_amd import dygrass as D

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    for flags in (0, BATCHED):
        wl = _rmat()
        o, d = make_pair(wl, variant=TWO, flags=flags)
        try:
            for t, b in enumerate(wl.batches):
                say(f"  two-stage dev batch {t} flags={flags}")
                ro = o.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, s=b.s, L=b.L)

                def T(a, dt):
                    return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)

                res = torch.zeros(b.size * 24, dtype=torch.uint8, device=dev)
                kw = dict(s=T(b.s.astype(np.int16), np.int16),
                          L=T(b.L.astype(np.int16), np.int16), L_max=int(b.L.max()),
                          s_max=int(b.s.max()), results=res)
                if t % 2:
                    kw["stream"] = stream
                D.dyg_apply_batch_dev(d.ctx, T(b.iu, np.int32), T(b.iv, np.int32),
                                      T(b.iw, np.float64), T(b.du, np.int32),
                                      T(b.dv, np.int32), **kw)
                D.dyg_sync(d.ctx)
                rl = res.cpu().numpy().view(D.UPDATE_RESULT_DTYPE)
                for key in ("flag", "any_hit", "winner", "n_rec", "steps"):
                    assert np.array_equal(rl[key], ro[key]), (t, key)
                assert np.array_equal(rl["Rmin"], ro["Rmin"])
                compare_state(o, d, f"two-stage dev {t}")
        finally:
            d.close()
            o.close()


def test_two_stage_refused_where_unsupported():
    from paper_2505_02741_amd import dygrass as D

    wl = W.make_workload("grid64", batches=1)
    with pytest.raises(D.DygError):
        make_pair(wl, variant=TWO, flags=BATCHED | D.FLAG_AUTOTUNE)
    o, d = make_pair(wl, variant=TWO)
    try:
        with D.DygServer() as srv, pytest.raises(D.DygError):
            srv.add_graph(d)
    finally:
        d.close()
        o.close()


def test_unweighted_selection_parity():
    """A reference weight of 1e300 quantises every weight to 1: the choice is
    uniform over the candidates, the unbiased neighbour choice of Sec. II-D."""
    run_parity(_mesh(), tag="uniform selection", w_ref=1e300)
    run_parity(_rmat(), tag="uniform selection batched", w_ref=1e300, flags=BATCHED)
