"""Batched form (work-queue walks) and the device-resident entry point, against
the CPU oracle element by element."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2505_02741_amd import workloads as W

from gpu_helpers import compare_batch, compare_state, make_pair, run_parity, say

pytestmark = pytest.mark.gpu

BATCHED = 4  # DYG_FLAG_BATCHED


def test_batched_grid64():
    wl = W.make_workload("grid64")
    run_parity(wl, tag="batched grid64", flags=BATCHED)


@pytest.mark.parametrize("K", [1.0, 4.0])
def test_batched_threshold(K):
    wl = W.make_workload("grid64", batches=3)
    run_parity(wl, tag=f"batched K={K}", K=K, flags=BATCHED)


def test_batched_mesh_fully_dynamic():
    wl = W.make_workload("mesh128", side=12, ins=150, dels=150, batches=6)
    run_parity(wl, tag="batched mesh12", flags=BATCHED)


def test_batched_uneven_walkers_and_limits():
    wl = W.make_workload("mesh128", side=10, ins=120, dels=120, batches=4)
    rng = np.random.default_rng(9)
    for b in wl.batches:
        b.s = rng.integers(0, 201, b.size).astype(np.uint16)
        b.L = rng.integers(0, 41, b.size).astype(np.uint16)
    run_parity(wl, tag="batched uneven", flags=BATCHED)


def test_batched_power_law():
    wl = W.make_workload("rmat22", scale=11, batches=4, size_lo=50, size_hi=800)
    run_parity(wl, tag="batched rmat11", flags=BATCHED)


def test_batched_bounce():
    wl = W.make_workload("grid64", side=24, ins=200, batches=3)
    run_parity(wl, tag="batched bounce", dead_end=1, flags=BATCHED)


@pytest.mark.parametrize("flags", [0, BATCHED])
def test_device_resident_batches(flags):
    """dyg_apply_batch_dev on torch tensors: same results as the oracle, on
    the library's stream and on a caller stream."""
    import torch

    from paper_2505_02741_amd import dygrass as D

    dev = torch.device("cuda:0")
    wl = W.make_workload("rmat22", scale=11, batches=4, size_lo=50, size_hi=800)
    o, d = make_pair(wl, flags=flags)
    stream = torch.cuda.Stream()
    try:
        for t, b in enumerate(wl.batches):
            say(f"  dev batch {t} flags={flags}")
            ro = o.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, s=b.s, L=b.L)

            def T(a, dt):
                return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)

            res = torch.zeros(b.size * 24, dtype=torch.uint8, device=dev)
            kw = dict(s=T(b.s.astype(np.int16), np.int16), L=T(b.L.astype(np.int16), np.int16),
                      L_max=int(b.L.max()), s_max=int(b.s.max()), results=res)
            if t % 2:
                kw["stream"] = stream
            D.dyg_apply_batch_dev(d.ctx, T(b.iu, np.int32), T(b.iv, np.int32),
                                  T(b.iw, np.float64), T(b.du, np.int32), T(b.dv, np.int32), **kw)
            D.dyg_sync(d.ctx)
            rl = res.cpu().numpy().view(D.UPDATE_RESULT_DTYPE)
            for key in ("flag", "any_hit", "winner", "n_rec", "steps"):
                assert np.array_equal(rl[key], ro[key]), (t, key)
            assert np.array_equal(rl["Rmin"], ro["Rmin"])
            compare_state(o, d, f"dev {t}")
    finally:
        d.close()
        o.close()


def test_device_batch_validation_error():
    import torch

    from paper_2505_02741_amd import dygrass as D

    dev = torch.device("cuda:0")
    wl = W.make_workload("grid64", side=8, ins=5, batches=1)
    o, d = make_pair(wl, flags=BATCHED)
    try:
        before = d.query("H")
        iu = torch.tensor([0], dtype=torch.int32, device=dev)
        iv = torch.tensor([0], dtype=torch.int32, device=dev)
        iw = torch.tensor([1.0], dtype=torch.float64, device=dev)
        z = torch.zeros(0, dtype=torch.int32, device=dev)
        D.dyg_apply_batch_dev(d.ctx, iu, iv, iw, z, z)
        with pytest.raises(D.DygError) as e:
            D.dyg_sync(d.ctx)
        assert e.value.name == "SELF_LOOP"
        for a, b_ in zip(before, d.query("H")):
            assert np.array_equal(a, b_)
        compare_batch(o, d, wl.batches[0], tag="after dev error")
        compare_state(o, d, "after dev error")
    finally:
        d.close()
        o.close()


GRAPH = 8  # DYG_FLAG_GRAPH


def _uneven_mesh_batches(seed=4):
    """Mesh batches of varying sizes: several size classes, each seen more than
    once, so captured graphs are both created and replayed."""
    wl = W.make_workload("mesh128", side=12, ins=10, dels=10, batches=0)
    es = W.EdgeSet(wl.G)
    rng = np.random.default_rng(seed)
    for size in (300, 40, 290, 35, 300, 9, 150, 41, 260, 8):
        n_ins = size // 2
        p, q = W.local_insertions_lattice(es, 12, 3, n_ins, rng, np.zeros(0, np.int64))
        du, dv = W.uniform_deletions(es, size - n_ins, rng)
        b = W.Batch(p.astype(np.uint32), q.astype(np.uint32), rng.uniform(0.5, 2.0, p.size),
                    du.astype(np.uint32), dv.astype(np.uint32))
        es.apply(es.key(b.iu, b.iv), es.key(b.du, b.dv))
        wl.batches.append(b)
    return wl


@pytest.mark.parametrize("flags", [GRAPH, BATCHED | GRAPH])
def test_graph_mode_replays(flags):
    wl = _uneven_mesh_batches()
    run_parity(wl, tag=f"graph flags={flags}", flags=flags)


def test_graph_mode_error_then_valid():
    from paper_2505_02741_amd import dygrass as D

    wl = _uneven_mesh_batches()
    o, d = make_pair(wl, flags=BATCHED | GRAPH)
    try:
        compare_batch(o, d, wl.batches[0], tag="graph b0")
        b = wl.batches[1]
        bad_iu = b.iu.copy()
        bad_iu[3] = b.iv[3]  # a self loop inside an otherwise valid batch
        with pytest.raises(D.DygError) as e:
            d.apply_batch(bad_iu, b.iv, b.iw, b.du, b.dv)
        assert e.value.name == "SELF_LOOP"
        compare_state(o, d, "graph after error")
        for t, bb in enumerate(wl.batches[1:]):
            compare_batch(o, d, bb, tag=f"graph b{t + 1}")
        compare_state(o, d, "graph end")
    finally:
        d.close()
        o.close()


@pytest.mark.parametrize("upw", [0, 1, 3, 8])
def test_walk_schedules_agree(upw):
    """The batched form's walk schedule (one work queue, or ranges of upw
    updates per wavefront) changes no result: uneven walker counts and step
    limits, insertions and deletions, against the oracle."""
    from paper_2505_02741_amd import dygrass as D

    wl = W.make_workload("mesh128", side=10, ins=150, dels=120, batches=4)
    rng = np.random.default_rng(17)
    for b in wl.batches:
        b.s = rng.integers(0, 150, b.size).astype(np.uint16)
        b.L = rng.integers(1, 30, b.size).astype(np.uint16)
    o, d = make_pair(wl, flags=BATCHED)
    try:
        D.dyg_set_tuning(d.ctx, 4, 1, upw, 0)
        for t, b in enumerate(wl.batches):
            compare_batch(o, d, b, tag=f"upw={upw} batch {t}")
        compare_state(o, d, f"upw={upw}")
        st = d.stats()
        assert st["walk_steps"] == o.steps_total
        assert st["walk_alg_bytes"] == o.alg_bytes_total
    finally:
        d.close()
        o.close()


@pytest.mark.parametrize("tail_lanes,upw", [(8, 1), (16, 4), (64, 8)])
def test_head_tail_schedule_agrees(tail_lanes, upw):
    """The head/tail schedule (lockstep head per update, survivors packed into
    tail wavefronts) changes no result: walker counts from 0 to 149 (rounds of
    64, heads too small to hand anything off), uneven step limits, insertions
    and deletions, against the oracle."""
    from paper_2505_02741_amd import dygrass as D

    wl = W.make_workload("mesh128", side=10, ins=150, dels=120, batches=4)
    rng = np.random.default_rng(23)
    for b in wl.batches:
        b.s = rng.integers(0, 150, b.size).astype(np.uint16)
        b.L = rng.integers(1, 30, b.size).astype(np.uint16)
    o, d = make_pair(wl, flags=BATCHED)
    try:
        D.dyg_set_tuning(d.ctx, 8, 1, upw, tail_lanes)
        assert D.dyg_get_tuning(d.ctx)["tail_lanes"] == tail_lanes
        for t, b in enumerate(wl.batches):
            compare_batch(o, d, b, tag=f"tail={tail_lanes} upw={upw} batch {t}")
        compare_state(o, d, f"tail={tail_lanes}")
        st = d.stats()
        assert st["walk_steps"] == o.steps_total
        assert st["walk_alg_bytes"] == o.alg_bytes_total
    finally:
        d.close()
        o.close()


def test_head_tail_schedule_hubs_and_graph_mode():
    """Head/tail schedule on a power-law graph (hub rows) and replayed from
    captured graphs: the oracle's results."""
    from paper_2505_02741_amd import dygrass as D

    wl = W.make_workload("rmat22", scale=11, batches=4, size_lo=50, size_hi=800)
    o, d = make_pair(wl, flags=BATCHED | GRAPH)
    try:
        D.dyg_set_tuning(d.ctx, 8, 1, 4, 16)
        for t, b in enumerate(wl.batches):
            compare_batch(o, d, b, tag=f"rmat head/tail batch {t}")
        compare_state(o, d, "rmat head/tail")
    finally:
        d.close()
        o.close()


@pytest.mark.parametrize("graph", [False, True])
def test_lockstep_schedule_in_the_batched_form(graph):
    """The batched form with the lockstep walk (one wavefront per update,
    decisions inside the walk kernel), launched directly or replayed from
    captured graphs, on a power-law graph with hub rows: the oracle's results,
    walker records included."""
    from paper_2505_02741_amd import dygrass as D

    wl = W.make_workload("rmat22", scale=11, batches=4, size_lo=50, size_hi=800)
    o, d = make_pair(wl, flags=BATCHED | (GRAPH if graph else 0))
    try:
        D.dyg_set_tuning(d.ctx, 8, 1, 4, 0, lockstep=1)
        assert D.dyg_get_tuning(d.ctx)["lockstep"] == 1
        for t, b in enumerate(wl.batches):
            compare_batch(o, d, b, tag=f"lockstep graph={graph} batch {t}")
        compare_state(o, d, f"lockstep graph={graph}")
        st = d.stats()
        assert st["walk_steps"] == o.steps_total
        assert st["walk_alg_bytes"] == o.alg_bytes_total
        with pytest.raises(D.DygError):
            D.dyg_set_tuning(d.ctx, 8, 1, 4, 0, lockstep=2)
    finally:
        d.close()
        o.close()


@pytest.mark.parametrize("flags", [0, BATCHED])
def test_reserved_buffers(flags):
    """dyg_reserve sizes the batch buffers up front; results stay the oracle's,
    and out-of-range bounds are refused."""
    from paper_2505_02741_amd import dygrass as D

    wl = W.make_workload("rmat22", scale=11, batches=4, size_lo=50, size_hi=800)
    o, d = make_pair(wl, flags=flags)
    try:
        D.dyg_reserve(d.ctx, 2000, 2000, 128, 32)
        with pytest.raises(D.DygError) as e:
            D.dyg_reserve(d.ctx, 10, 10, 5000, 8)
        assert e.value.name == "INVALID_ARG"
        for t, b in enumerate(wl.batches):
            compare_batch(o, d, b, tag=f"reserved {t}")
        compare_state(o, d, "reserved")
    finally:
        d.close()
        o.close()


def test_autotune_keeps_results_and_picks_a_schedule():
    """With DYG_FLAG_AUTOTUNE the first batches each run another walk
    schedule; every batch still matches the oracle, and after the trials the
    context keeps one of the candidates."""
    from paper_2505_02741_amd import dygrass as D

    wl = W.make_workload("mesh128", side=10, ins=120, dels=100, batches=12)
    o, d = make_pair(wl, flags=BATCHED | D.FLAG_AUTOTUNE)
    try:
        for t, b in enumerate(wl.batches):
            compare_batch(o, d, b, record=False, tag=f"autotune {t}")
        compare_state(o, d, "autotune")
        t = D.dyg_get_tuning(d.ctx)
        say("  kept schedule:", t)
        assert t["updates_per_wave"] in (0, 1, 2, 4, 8)
        assert t["tail_lanes"] in (0, 8, 16)
        assert t["lockstep"] in (0, 1)
        assert d.stats()["walk_launches"] >= 10  # the trials were timed
    finally:
        d.close()
        o.close()
