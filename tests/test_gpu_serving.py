"""Serving form (dyg_server_*): many resident graphs, requests fused into
shared launches.  Every request's results, and every graph's final edge sets,
must equal what the CPU oracle gives for that graph's own request stream
applied alone and in order, whatever else shares the launch."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2505_02741_amd import workloads as W

from gpu_helpers import close_R, compare_state, make_pair, say

pytestmark = pytest.mark.gpu

BATCHED = 4


def _fleet():
    """Small graphs of different kinds and sizes, each with its own stream."""
    return [
        W.make_workload("grid64", seed=1, side=20, ins=60, batches=4),
        W.make_workload("mesh128", seed=2, side=8, ins=40, dels=40, batches=4),
        W.make_workload("grid64", seed=3, side=28, ins=150, batches=3),
        W.make_workload("rmat22", seed=4, scale=10, batches=4, size_lo=20, size_hi=300),
        W.make_workload("mesh128", seed=5, side=10, ins=90, dels=70, batches=5),
        W.make_workload("grid64", seed=6, side=12, ins=5, batches=6),
    ]


def _oracle_stream(o, batches):
    # the server walks every update with the graph's default s and L
    return [o.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv) for b in batches]


def _check(res, ro, tag):
    for key in ("flag", "any_hit", "winner", "n_rec", "steps"):
        bad = np.flatnonzero(res[key] != ro[key])
        assert bad.size == 0, f"{tag} {key} differs at {bad[:8]}"
    assert close_R(res["Rmin"], ro["Rmin"]), tag


def _interleave(counts, rng):
    """A random submission order that keeps each graph's own order."""
    left = list(counts)
    nxt = [0] * len(counts)
    order = []
    while any(left):
        g = int(rng.choice([i for i, k in enumerate(left) if k]))
        order.append((g, nxt[g]))
        nxt[g] += 1
        left[g] -= 1
    return order


@pytest.mark.parametrize("max_fused,max_inflight,mem_budget",
                         [(8, 2, 8 << 30), (3, 1, 8 << 30), (16, 3, 1 << 20)])
def test_serving_equals_each_graph_alone(max_fused, max_inflight, mem_budget):
    from paper_2505_02741_amd import dygrass as D

    wls = _fleet()
    pairs = [make_pair(wl, flags=BATCHED) for wl in wls]
    try:
        expect = [_oracle_stream(o, wl.batches) for (o, _), wl in zip(pairs, wls)]
        order = _interleave([len(wl.batches) for wl in wls], np.random.default_rng(11))
        with D.DygServer(mem_budget=mem_budget, max_fused=max_fused,
                         max_inflight=max_inflight) as srv:
            gids = [srv.add_graph(d) for _, d in pairs]
            owner = {}
            done = []
            for k, (g, t) in enumerate(order):
                b = wls[g].batches[t]
                rid = srv.submit(gids[g], b.iu, b.iv, b.iw, b.du, b.dv)
                owner[rid] = (g, t)
                if k % 3 == 2:
                    done += srv.poll()
            done += srv.drain()
        say(f"  served {len(done)} requests (fused<={max_fused}, inflight<={max_inflight})")
        assert sorted(owner) == sorted(r["request_id"] for r in done)
        finished_order = {g: [] for g in range(len(wls))}
        for r in done:
            g, t = owner[r["request_id"]]
            assert r["status"] == 0, (g, t, D.STATUS.get(r["status"]))
            assert r["graph_id"] == gids[g]
            assert r["n_updates"] == wls[g].batches[t].size
            assert r["t_submit"] <= r["t_start"] <= r["t_done"]
            _check(r["results"], expect[g][t], f"graph {g} batch {t}")
            finished_order[g].append(t)
        for g, ts in finished_order.items():
            assert ts == sorted(ts), f"graph {g} finished out of order: {ts}"
        for g, (o, d) in enumerate(pairs):
            compare_state(o, d, f"served graph {g}")
            assert d.stats()["uid_base"] == o.uid_base
    finally:
        for o, d in pairs:
            d.close()
            o.close()


def test_serving_bad_request_leaves_its_graph_and_the_others_intact():
    from paper_2505_02741_amd import dygrass as D

    wls = _fleet()[:4]
    pairs = [make_pair(wl, flags=BATCHED) for wl in wls]
    try:
        expect = [_oracle_stream(o, wl.batches) for (o, _), wl in zip(pairs, wls)]
        with D.DygServer(max_fused=8, max_inflight=2) as srv:
            gids = [srv.add_graph(d) for _, d in pairs]
            owner = {}
            for t in range(3):
                for g, wl in enumerate(wls):
                    b = wl.batches[t]
                    if g == 1 and t == 1:
                        # a deletion of an edge that is not in G, between two
                        # good requests of the same graph
                        bad = srv.submit(gids[g], b.iu, b.iv, b.iw,
                                         np.r_[b.du, np.uint32(0)], np.r_[b.dv, np.uint32(0)])
                        owner[bad] = (g, -1)
                    rid = srv.submit(gids[g], b.iu, b.iv, b.iw, b.du, b.dv)
                    owner[rid] = (g, t)
            done = srv.drain()
        for r in done:
            g, t = owner[r["request_id"]]
            if t < 0:
                assert D.STATUS[r["status"]] in ("SELF_LOOP", "EDGE_MISSING"), r["status"]
                continue
            assert r["status"] == 0, (g, t, D.STATUS.get(r["status"]))
            _check(r["results"], expect[g][t], f"graph {g} batch {t}")
        for g, (o, d) in enumerate(pairs):
            # the oracle applied batches 0..3; the server only 0..2
            o2, _ = make_pair(wls[g], flags=BATCHED)
            _.close()
            for b in wls[g].batches[:3]:
                o2.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv)
            compare_state(o2, d, f"graph {g} after bad request")
            o2.close()
    finally:
        for o, d in pairs:
            d.close()
            o.close()


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_serving_fleet_with_a_two_million_vertex_graph():
    """A fleet at the serving configuration's sizes: a 1448x1448 grid (about
    2.1M vertices), a 3D mesh of 64^3, an R-MAT graph of scale 17 and two
    small graphs, with requests of up to 50,000 updates (60% insertions)
    fused across graphs; every request's results and every graph's final
    edge sets against the oracle run on that graph's stream alone."""
    from paper_2505_02741_amd import dygrass as D

    over = dict(size_lo=1, ins_frac=0.6, s=64, L=24)
    wls = [
        W.make_workload("grid1024", seed=21, side=1448, batches=3, size_hi=50_000, **over),
        W.make_workload("mesh128", seed=22, side=64, batches=3, size_hi=50_000, **over),
        W.make_workload("rmat22", seed=23, scale=17, batches=3, size_hi=50_000, s_lo=None,
                        s_hi=None, L_lo=None, L_hi=None, **over),
        W.make_workload("grid64", seed=24, side=100, batches=4, size_hi=2_000, **over),
        W.make_workload("mesh128", seed=25, side=16, batches=4, size_hi=1_000, **over),
    ]
    say(f"  fleet: {[wl.G.n for wl in wls]} vertices, "
        f"{[[b.size for b in wl.batches] for wl in wls]} updates")
    assert max(wl.G.n for wl in wls) >= 2_000_000
    pairs = [make_pair(wl, flags=BATCHED) for wl in wls]
    try:
        expect = [_oracle_stream(o, wl.batches) for (o, _), wl in zip(pairs, wls)]
        say("  oracle streams done")
        order = _interleave([len(wl.batches) for wl in wls], np.random.default_rng(5))
        with D.DygServer(mem_budget=16 << 30, max_fused=8, max_inflight=2) as srv:
            gids = [srv.add_graph(d) for _, d in pairs]
            owner = {}
            for g, t in order:
                b = wls[g].batches[t]
                owner[srv.submit(gids[g], b.iu, b.iv, b.iw, b.du, b.dv)] = (g, t)
            done = srv.drain()
        assert sorted(owner) == sorted(r["request_id"] for r in done)
        for r in done:
            g, t = owner[r["request_id"]]
            assert r["status"] == 0, (g, t, D.STATUS.get(r["status"]))
            _check(r["results"], expect[g][t], f"graph {g} batch {t}")
        for g, (o, d) in enumerate(pairs):
            compare_state(o, d, f"served graph {g}")
        say(f"  served {len(done)} requests, all equal to the oracle")
    finally:
        for o, d in pairs:
            d.close()
            o.close()
