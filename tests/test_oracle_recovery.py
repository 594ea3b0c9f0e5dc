"""Pins of the oracle's deletion repair: the recovered path and the no-hit
fallback (Sec. III-C; Algorithm 1, deletion branch), on hand-built graphs
whose answers are computed by hand or follow from the graph's structure.

* The recovered edges are those of the hitting walker of least resistance
  (Eq. 12), in path order, each once, leaving out edges already in H.
* With no hit, each endpoint recovers its G edge of least resistance (largest
  weight) that is not in H, ties to the smaller neighbour id: a reading of
  the paper's local fallback, which the paper does not define further.

Each case asserts the exact recovered edge list, its order, n_rec, the winner
and the final H.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from paper_2505_02741_amd import workloads as W


def _oracle(oracle_mod, n, edges, h_edges, *, s=8, L=16, seed=11, uid_base=0):
    u = np.array([a for a, _, _ in edges], dtype=np.uint32)
    v = np.array([b for _, b, _ in edges], dtype=np.uint32)
    w = np.array([x for _, _, x in edges], dtype=np.float64)
    rp, col, ww = W.to_csr(n, u, v, w)
    hu = np.array([a for a, _ in h_edges], dtype=np.uint32)
    hv = np.array([b for _, b in h_edges], dtype=np.uint32)
    return oracle_mod.Oracle(n, rp, col, ww, hu, hv, seed=seed, s=s, L=L, uid_base=uid_base)


def _H(o):
    u, v, _ = o.query("H")
    return {(int(a), int(b)) for a, b in zip(u, v)}


def _key(a, b):
    return (min(a, b), max(a, b))


def _delete(o, pairs, record=True):
    z = np.zeros(0)
    du = [a for a, _ in pairs]
    dv = [b for _, b in pairs]
    return o.apply_batch(z, z, z, du, dv, record_walkers=record)


# --------------------------------------------------------------------------
# a deterministic path: every walker follows the same route


CYCLE_W = [1.0 + 0.5 * i for i in range(8)]  # weight of edge (i, i+1)


def _cycle(oracle_mod, L):
    edges = [(i, i + 1, CYCLE_W[i]) for i in range(8)] + [(0, 8, 2.0)]
    h = [(0, 8), (0, 1), (1, 2), (4, 5)]
    return _oracle(oracle_mod, 9, edges, h, s=4, L=L)


def test_cycle_recovers_path_edges_not_in_H_in_path_order(oracle_mod):
    """Deleting (0,8) from a 9-cycle leaves a path: every walker goes
    0,1,...,8 and hits at step 8 with the same R, so walker 0 wins and the
    path edges outside H are recovered in path order."""
    o = _cycle(oracle_mod, L=12)
    r = _delete(o, [(0, 8)])
    assert r["flag"][0] == 1 and r["any_hit"][0] == 1
    assert r["winner"][0] == 0
    R = 0.0
    for x in CYCLE_W:
        R = R + 1.0 / x
    assert r["Rmin"][0] == R
    assert list(r["walkers"]["steps"]) == [8] * 4 and list(r["walkers"]["hit"]) == [1] * 4
    assert o.last_recovered(0) == [(2, 3), (3, 4), (5, 6), (6, 7), (7, 8)]
    assert r["n_rec"][0] == 5
    assert _H(o) == {(0, 1), (1, 2), (4, 5), (2, 3), (3, 4), (5, 6), (6, 7), (7, 8)}


def test_cycle_recovery_from_the_other_endpoint(oracle_mod):
    """The same deletion given as (8,0): the walk runs 8,7,...,0 and the
    recovered edges come in that order, oriented along the walk."""
    o = _cycle(oracle_mod, L=12)
    r = _delete(o, [(8, 0)])
    assert r["any_hit"][0] == 1 and r["winner"][0] == 0
    assert o.last_recovered(0) == [(8, 7), (7, 6), (6, 5), (4, 3), (3, 2)]
    assert r["n_rec"][0] == 5


def test_cycle_too_short_a_walk_takes_the_fallback(oracle_mod):
    """With L = 5 no walker reaches 8.  Fallback: vertex 0's only G edge,
    (0,1), is in H, so 0 adds nothing; vertex 8's only G edge (8,7) is not
    in H and is recovered."""
    o = _cycle(oracle_mod, L=5)
    r = _delete(o, [(0, 8)])
    assert r["any_hit"][0] == 0 and r["winner"][0] == 0xFFFF and math.isinf(r["Rmin"][0])
    assert o.last_recovered(0) == [(8, 7)]
    assert r["n_rec"][0] == 1
    assert _H(o) == {(0, 1), (1, 2), (4, 5), (7, 8)}


# --------------------------------------------------------------------------
# two routes of different resistance: the least-resistance hit wins


def _two_route_gadgets(oracle_mod, count, s=8):
    """count disjoint copies of: u=0, v=5, route A 0-1-2-5 (R = 1 + 1/4 + 1/4
    = 1.5), route B 0-3-4-5 (R = 1 + 1 + 1 = 3), both first edges of weight 1
    (equally likely), and the edge (0,5) that is deleted."""
    edges, h = [], []
    for g in range(count):
        b = 6 * g
        edges += [(b, b + 1, 1.0), (b + 1, b + 2, 4.0), (b + 2, b + 5, 4.0),
                  (b, b + 3, 1.0), (b + 3, b + 4, 1.0), (b + 4, b + 5, 1.0), (b, b + 5, 1.0)]
        h += [(b, b + 5), (b, b + 1), (b, b + 3), (b + 4, b + 5)]
    return _oracle(oracle_mod, 6 * count, edges, h, s=s, L=10)


def test_least_resistance_route_is_recovered(oracle_mod):
    count, s = 16, 8
    o = _two_route_gadgets(oracle_mod, count, s)
    r = _delete(o, [(6 * g, 6 * g + 5) for g in range(count)])
    wk = r["walkers"]
    walker0_on_B = 0
    for g in range(count):
        b = 6 * g
        R = wk["R"][g * s:(g + 1) * s]
        # every walker hits in three steps along one of the two routes
        assert set(R.tolist()) <= {1.5, 3.0} and np.all(wk["hit"][g * s:(g + 1) * s] == 1)
        assert 1.5 in R.tolist(), "precondition: some walker took route A"
        walker0_on_B += int(R[0] == 3.0)
        assert r["Rmin"][g] == 1.5
        assert r["winner"][g] == int(np.flatnonzero(R == 1.5)[0])
        # route A's edges outside H, in path order
        assert o.last_recovered(g) == [(b + 1, b + 2), (b + 2, b + 5)]
        assert r["n_rec"][g] == 2
    # precondition: the first walker is not always the winner
    assert walker0_on_B > 0
    expect = set()
    for g in range(count):
        b = 6 * g
        expect |= {(b, b + 1), (b, b + 3), (b + 4, b + 5), (b + 1, b + 2), (b + 2, b + 5)}
    assert _H(o) == expect


# --------------------------------------------------------------------------
# no hit: the fallback, hand computed


def test_fallback_largest_weight_not_in_H_ties_to_smaller_id(oracle_mod):
    """(0,9) is a bridge: after its deletion no walker from 0 can reach 9.
    Vertex 0's G edges: 1 (w 2, in H), 2 (w 5), 3 (w 5), 4 (w 1) -> the tie
    at w 5 goes to the smaller id, (0,2).  Vertex 9's: 5 (w 0.5), 6 (w 3),
    7 (w 3), 8 (w 3.5, in H) -> (9,6).  A second bridge (10,13) in another
    component: vertex 10's only other edge (10,11) is in H, so only 13
    contributes its heavier edge (13,12)."""
    edges = [(0, 1, 2.0), (0, 2, 5.0), (0, 3, 5.0), (0, 4, 1.0), (1, 2, 1.5),
             (5, 9, 0.5), (6, 9, 3.0), (7, 9, 3.0), (8, 9, 3.5), (6, 7, 1.0), (0, 9, 1.0),
             (10, 11, 1.0), (10, 13, 1.0), (12, 13, 4.0), (13, 14, 2.0), (12, 14, 1.0)]
    h = [(0, 9), (0, 1), (8, 9), (10, 13), (10, 11), (12, 14)]
    o = _oracle(oracle_mod, 15, edges, h, s=8, L=6)
    r = _delete(o, [(0, 9), (10, 13)])
    assert list(r["any_hit"]) == [0, 0]
    assert list(r["flag"]) == [1, 1]
    assert list(r["winner"]) == [0xFFFF, 0xFFFF]
    assert o.last_recovered(0) == [(0, 2), (9, 6)]
    assert o.last_recovered(1) == [(13, 12)]
    assert list(r["n_rec"]) == [2, 1]
    assert _H(o) == {(0, 1), (8, 9), (10, 11), (12, 14), (0, 2), (6, 9), (12, 13)}


def test_single_step_deletion_cannot_hit(oracle_mod):
    """Square 0-1-2-3 with L = 1: after one step a walker from 0 stands on 3
    (the deleted edge (0,1) is gone), so nobody hits; the fallback adds each
    endpoint's only remaining edge, (0,3) and (1,2)."""
    edges = [(0, 1, 1.0), (1, 2, 2.0), (2, 3, 3.0), (0, 3, 4.0)]
    o = _oracle(oracle_mod, 4, edges, [(0, 1), (2, 3)], s=4, L=1)
    r = _delete(o, [(0, 1)])
    assert r["any_hit"][0] == 0
    assert list(r["walkers"]["steps"]) == [1] * 4 and list(r["walkers"]["end"]) == [3] * 4
    assert o.last_recovered(0) == [(0, 3), (1, 2)]
    assert _H(o) == {(2, 3), (0, 3), (1, 2)}


# --------------------------------------------------------------------------
# a resistance sum that overflows still names its walker


def test_infinite_resistance_hit_still_wins(oracle_mod):
    """Weights of 1e-308 have 1/w = 1e308 (finite); two of them sum to +inf.
    Deleting (0,3) from the 4-cycle leaves the path 0-1-2-3: every walker
    hits at step 3 with R = +inf, so walker 0 wins and the path is
    recovered."""
    tiny = 1e-308
    assert math.isfinite(1.0 / tiny)
    edges = [(0, 1, tiny), (1, 2, tiny), (2, 3, tiny), (0, 3, 1.0)]
    o = _oracle(oracle_mod, 4, edges, [(0, 3)], s=4, L=8)
    r = _delete(o, [(0, 3)])
    assert r["any_hit"][0] == 1
    assert math.isinf(r["Rmin"][0])
    assert r["winner"][0] == 0
    assert o.last_recovered(0) == [(0, 1), (1, 2), (2, 3)]
    assert r["n_rec"][0] == 3


def test_weight_with_infinite_resistance_is_rejected(oracle_mod):
    """1/w of a weight below about 5.6e-309 overflows: such a weight is
    refused at init and in a batch (BAD_WEIGHT)."""
    bad = 1e-310
    assert math.isinf(1.0 / bad)
    with pytest.raises(oracle_mod.OracleError) as ei:
        _oracle(oracle_mod, 3, [(0, 1, 1.0), (1, 2, bad)], [])
    assert ei.value.name == "BAD_WEIGHT"
    o = _oracle(oracle_mod, 3, [(0, 1, 1.0), (1, 2, 1.0)], [])
    z = np.zeros(0)
    with pytest.raises(oracle_mod.OracleError) as ei:
        o.apply_batch([0], [2], [bad], z, z)
    assert ei.value.name == "BAD_WEIGHT"


# --------------------------------------------------------------------------
# random graphs with short cycles: the rule restated against the trajectories


def _winner_path_edges(tr, steps):
    return [(int(tr[t]), int(tr[t + 1])) for t in range(steps)]


@pytest.mark.parametrize("seed,s", [(3, 4), (8, 4), (6, 64)])
def test_recovered_list_follows_the_rule_on_cyclic_graphs(oracle_mod, seed, s):
    """A 6x6 grid with random chords, H its maximum spanning forest plus a
    few edges; a batch deletes several H edges.  For every deletion the
    walks on the batch snapshot G_mid (the static-graph walk, pinned
    separately) give the trajectories; the expected list is the least-R
    hitter's path, first occurrence of each edge, without H_mid's edges.
    With few walkers some winning path repeats an edge (so the first-
    occurrence rule is exercised); with many, the winner is picked among
    many hits."""
    rng = np.random.default_rng(seed)
    n, u, v = W.grid2d(6)
    chords = rng.choice(n, (14, 2))
    u = np.concatenate([u, chords[:, 0]]).astype(np.int64)
    v = np.concatenate([v, chords[:, 1]]).astype(np.int64)
    u, v = W._canonical(n, u, v)
    w = rng.uniform(0.5, 3.0, u.size)
    mask = W.max_spanning_forest(n, u, v, w)
    mask[rng.choice(np.flatnonzero(~mask), 6, replace=False)] = True
    edges = list(zip(u.tolist(), v.tolist(), w.tolist()))
    h = [(a, b) for (a, b, _), m in zip(edges, mask) if m]
    L = 40
    o = _oracle(oracle_mod, n, edges, h, s=s, L=L, seed=1000 + seed)
    hidx = np.flatnonzero(mask)
    pick = rng.choice(hidx, 8, replace=False)
    dels = [(int(u[e]), int(v[e])) if rng.random() < 0.5 else (int(v[e]), int(u[e]))
            for e in pick]
    dkeys = {_key(a, b) for a, b in dels}
    H_mid = {_key(a, b) for a, b in h} - dkeys
    keep = np.array([_key(a, b) not in dkeys for a, b, _ in edges])
    rp, col, ww = W.to_csr(n, u[keep], v[keep], w[keep])
    w_ref = float(w.max())
    r = _delete(o, dels)
    repeats = 0
    for j, (a, b) in enumerate(dels):
        wk = oracle_mod.walk_csr(n, rp, col, ww, a, b, s=s, L=L, seed=1000 + seed, uid=j,
                                 w_ref=w_ref)
        hits = np.flatnonzero(wk["hit"])
        if hits.size == 0:
            continue
        # least R, ties to the lower walker index
        best = min(hits.tolist(), key=lambda k: (wk["R"][k], k))
        assert r["winner"][j] == best
        path = _winner_path_edges(wk["traj"][best], int(wk["steps"][best]))
        seen, expect = set(), []
        for x, y in path:
            k = _key(x, y)
            if k in seen:
                repeats += int(k not in H_mid)
                continue
            seen.add(k)
            if k not in H_mid:
                expect.append((x, y))
        assert o.last_recovered(j) == expect, j
        assert r["n_rec"][j] == len(expect)
    if s <= 4:
        assert repeats > 0, "precondition: some winning path repeats an edge outside H"
