"""Failure and edge paths through the C ABI on the GPU, against the oracle:
a hit whose resistance sum overflows, weights whose 1/w overflows, a pool
shortfall in a device-array batch (repaired at dyg_sync), and a serving
engine whose graph can no longer grow its pool (its waiting requests must
finish with an error and drain() must return).  Every failure is forced from
the host (a flag that makes pool growth fail); no kernel faults or hangs."""
from __future__ import annotations

import math
import time

import numpy as np
import pytest

from paper_2505_02741_amd import workloads as W

from gpu_helpers import compare_batch, compare_state, make_pair, say

pytestmark = pytest.mark.gpu

BATCHED = 4


def _tiny_weight_workload():
    """A 4-cycle 0-1-2-3 whose path edges weigh 1e-308 (1/w = 1e308), so a
    walker that goes round after (0,3) is deleted sums to +inf, plus a few
    disjoint copies so that several updates run."""
    tiny = 1e-308
    us, vs, ws = [], [], []
    for g in range(6):
        b = 4 * g
        for a, c, x in ((0, 1, tiny), (1, 2, tiny), (2, 3, tiny), (0, 3, 1.0)):
            us.append(b + a)
            vs.append(b + c)
            ws.append(x)
    n = 24
    u, v = np.array(us, np.uint32), np.array(vs, np.uint32)
    order = np.lexsort((v, u))
    G = W.Graph(n, u[order], v[order], np.array(ws)[order])
    h_mask = (G.v - G.u) == 3  # the edges (b, b+3)
    return W.Workload("tiny", G, h_mask, [], seed_walk=5, s=8, L=6)


@pytest.mark.parametrize("flags", [0, BATCHED], ids=["plain", "batched"])
def test_overflowing_resistance_hit_names_its_walker(flags):
    wl = _tiny_weight_workload()
    o, d = make_pair(wl, flags=flags)
    try:
        z = np.zeros(0, np.uint32)
        du = np.array([4 * g for g in range(6)], np.uint32)
        dv = du + 3
        b = W.Batch(z, z, np.zeros(0), du, dv)
        ro, rl = compare_batch(o, d, b, tag="inf R")
        assert np.all(rl["any_hit"] == 1) and np.all(np.isinf(rl["Rmin"]))
        assert np.all(rl["winner"] == 0) and np.all(rl["n_rec"] == 3)
        compare_state(o, d, "inf R")
    finally:
        d.close()
        o.close()


def test_weight_with_overflowing_resistance_is_rejected():
    from paper_2505_02741_amd import dygrass as D

    bad = 1e-310
    assert math.isinf(1.0 / bad)
    rp, col, w = W.to_csr(3, np.array([0, 1]), np.array([1, 2]), np.array([1.0, bad]))
    with pytest.raises(D.DygError) as ei:
        D.Dygrass(3, rp, col, w, [], [], seed=1)
    assert ei.value.code == -4
    rp, col, w = W.to_csr(3, np.array([0, 1]), np.array([1, 2]), np.array([1.0, 1.0]))
    d = D.Dygrass(3, rp, col, w, [], [], seed=1)
    try:
        z = np.zeros(0)
        with pytest.raises(D.DygError) as ei:
            d.apply_batch([0], [2], [bad], z, z)
        assert ei.value.code == -4
        assert d.stats()["uid_base"] == 0
    finally:
        d.close()


def _star_batches(wl, count=3, seed=1):
    """Insertions around a few centres: with zero slack and lean pools their
    rows overflow and the relocations exhaust the pool."""
    n = wl.G.n
    rng = np.random.default_rng(seed)
    es = W.EdgeSet(wl.G)
    out = []
    for _ in range(count):
        p = np.repeat(rng.choice(n, 4, replace=False), 60)
        q = rng.integers(0, n, p.size)
        k = es.key(p, q)
        ok = (p != q) & ~es.contains(k)
        _, first = np.unique(k[ok], return_index=True)
        sel = np.flatnonzero(ok)[np.sort(first)]
        p, q = p[sel], q[sel]
        out.append(W.Batch(p.astype(np.uint32), q.astype(np.uint32), rng.uniform(1, 10, p.size),
                           np.zeros(0, np.uint32), np.zeros(0, np.uint32)))
        es.apply(es.key(p, q), np.zeros(0, np.int64))
    return out


def test_pool_growth_in_a_device_batch_is_finished_at_sync():
    """The same shortfall as the host-array path, but the batch is enqueued
    from device arrays: dyg_sync must grow the pool, finish phase 4 and
    report success, and the state must equal the oracle's."""
    import torch

    from paper_2505_02741_amd import dygrass as D

    dev = torch.device("cuda:0")
    wl = W.make_workload("grid64", side=16, ins=0, batches=0)
    batches = _star_batches(wl)
    o, d = make_pair(wl, slack=0.0, s=8, L=6, flags=D.FLAG_LEAN_POOLS)
    try:
        for t, b in enumerate(batches):
            ro = o.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv)

            def T(a, dt):
                return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)

            res = torch.zeros(b.size * 24, dtype=torch.uint8, device=dev)
            D.dyg_apply_batch_dev(d.ctx, T(b.iu, np.int32), T(b.iv, np.int32),
                                  T(b.iw, np.float64), T(b.du, np.int32), T(b.dv, np.int32),
                                  results=res)
            D.dyg_sync(d.ctx)
            rl = res.cpu().numpy().view(D.UPDATE_RESULT_DTYPE)
            for key in ("flag", "any_hit", "steps"):
                assert np.array_equal(rl[key], ro[key]), (t, key)
            compare_state(o, d, f"device growth {t}")
        st = d.stats()
        say("  stats", st)
        assert st["compactions"] > 0 and st["uid_base"] == o.uid_base
    finally:
        d.close()
        o.close()


def test_failed_pool_growth_fails_the_batch_and_later_ones():
    from paper_2505_02741_amd import dygrass as D

    wl = W.make_workload("grid64", side=16, ins=0, batches=0)
    batches = _star_batches(wl)
    _, d = make_pair(wl, slack=0.0, s=8, L=6,
                     flags=D.FLAG_LEAN_POOLS | D.FLAG_FAIL_POOL_GROWTH)
    try:
        codes = []
        for b in batches:
            try:
                d.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv)
                codes.append(0)
            except D.DygError as e:
                codes.append(e.code)
        # the first batch that runs short fails, and so does every later one
        first = next(i for i, c in enumerate(codes) if c)
        assert all(c == -9 for c in codes[first:]), codes
    finally:
        d.close()


def test_server_drains_when_a_graph_cannot_grow_its_pool():
    """Graph 0 cannot grow its pool: its first request that runs short fails
    and its waiting requests finish with DYG_E_NOMEM at once; graph 1 is
    unaffected and matches the oracle; drain() returns."""
    from paper_2505_02741_amd import dygrass as D

    wl0 = W.make_workload("grid64", side=16, ins=0, batches=0)
    wl0.s, wl0.L = 8, 6
    stars = _star_batches(wl0, count=4)
    wl1 = W.make_workload("grid64", seed=2, side=20, ins=60, batches=4)
    _, d0 = make_pair(wl0, slack=0.0,
                      flags=BATCHED | D.FLAG_LEAN_POOLS | D.FLAG_FAIL_POOL_GROWTH)
    o1, d1 = make_pair(wl1, flags=BATCHED)
    srv = D.DygServer(max_fused=4, max_inflight=1)
    try:
        g0, g1 = srv.add_graph(d0), srv.add_graph(d1)
        ids0 = [srv.submit(g0, b.iu, b.iv, b.iw, b.du, b.dv) for b in stars]
        ids1 = [srv.submit(g1, b.iu, b.iv, b.iw, b.du, b.dv) for b in wl1.batches]
        done = []
        t_end = time.time() + 60
        while srv.pending and time.time() < t_end:
            done += srv.poll()
        assert srv.pending == 0, "drain did not finish"
        st = {r["request_id"]: r for r in done}
        codes0 = [st[i]["status"] for i in ids0]
        say("  graph 0 statuses", codes0)
        first = next(i for i, c in enumerate(codes0) if c)
        assert all(c == -9 for c in codes0[first:]), codes0
        for i, b in zip(ids1, wl1.batches):
            r = st[i]
            assert r["status"] == 0
            ro = o1.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv)
            for key in ("flag", "any_hit", "winner", "n_rec", "steps"):
                assert np.array_equal(r["results"][key], ro[key]), key
        compare_state(o1, d1, "unaffected graph")
    finally:
        srv.close()
        d0.close()
        d1.close()
        o1.close()
