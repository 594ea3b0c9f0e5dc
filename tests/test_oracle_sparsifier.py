"""Pins of the oracle's initial-sparsifier rule (maximum spanning forest by
Kruskal with ties to the smaller edge index, plus the off-tree edges of
smallest Philox sample key), each against something other than the oracle:
scipy's spanning tree, brute force over every spanning forest of tiny
graphs, the input generator's own Kruskal, and the sampling statistics."""
from __future__ import annotations

import itertools

import numpy as np
import pytest

from paper_2505_02741_amd import workloads as W


def _csr(n, u, v, w):
    return W.to_csr(n, np.asarray(u, np.uint32), np.asarray(v, np.uint32),
                    np.asarray(w, np.float64))


def _random_graph(rng, n, m_target, weights):
    pairs = set()
    while len(pairs) < m_target:
        a, b = rng.integers(0, n, 2)
        if a != b:
            pairs.add((min(a, b), max(a, b)))
    pairs = sorted(pairs)
    u = np.array([p[0] for p in pairs], np.uint32)
    v = np.array([p[1] for p in pairs], np.uint32)
    return u, v, weights(len(pairs))


def _components(n, u, v):
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for a, b in zip(u.tolist(), v.tolist()):
        parent[find(a)] = find(b)
    return len({find(x) for x in range(n)})


def test_forest_matches_scipy_on_distinct_weights(oracle_mod):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree

    rng = np.random.default_rng(3)
    for trial in range(5):
        n = 300
        u, v, w = _random_graph(rng, n, 700, lambda m: rng.uniform(1, 10, m))
        flags = oracle_mod.initial_sparsifier(n, *_csr(n, u, v, w), 0, 1)
        T = minimum_spanning_tree(csr_matrix((-w, (u.astype(np.int64), v.astype(np.int64))),
                                             shape=(n, n))).tocoo()
        want = {(min(a, b), max(a, b)) for a, b in zip(T.row.tolist(), T.col.tolist())}
        got = {(a, b) for a, b in zip(u[flags].tolist(), v[flags].tolist())}
        assert got == want, trial
        assert flags.sum() == n - _components(n, u, v)


def test_forest_is_the_greedy_optimum_under_ties_by_brute_force(oracle_mod):
    """With weights in {1, 2} many spanning forests have the maximum weight;
    the one Kruskal keeps under (weight descending, index ascending) is the
    spanning forest whose edge ranks, sorted, are lexicographically least
    (the greedy optimum of a matroid), found here by enumerating all."""
    rng = np.random.default_rng(5)
    for trial in range(12):
        n = 6
        u, v, w = _random_graph(rng, n, 9, lambda m: rng.integers(1, 3, m).astype(float))
        m = u.size
        c = _components(n, u, v)
        rank = {e: r for r, e in enumerate(sorted(range(m), key=lambda e: (-w[e], e)))}
        best = None
        for sub in itertools.combinations(range(m), n - c):
            if _components(n, u[list(sub)], v[list(sub)]) != c:
                continue  # not spanning (so a cycle)
            key = sorted(rank[e] for e in sub)
            if best is None or key < best[0]:
                best = (key, set(sub))
        flags = oracle_mod.initial_sparsifier(n, *_csr(n, u, v, w), 0, 1)
        assert set(np.flatnonzero(flags).tolist()) == best[1], trial


@pytest.mark.parametrize("name,over", [("grid64", dict(side=40)), ("mesh128", dict(side=9)),
                                       ("rmat22", dict(scale=11))])
def test_forest_equals_the_generators_kruskal(oracle_mod, name, over):
    """Two independent Kruskals: the input generator's (Python, ties by edge
    index) and the oracle's (C) keep the same forest; the generator lists
    edges in the same canonical (u, v) order."""
    wl = W.make_workload(name, batches=0, **over)
    g = wl.G
    want = W.max_spanning_forest(g.n, g.u, g.v, g.w)
    flags = oracle_mod.initial_sparsifier(g.n, *W.to_csr(g.n, g.u, g.v, g.w), 0, 1)
    cu, cv, _ = oracle_mod.canonical_edges(g.n, *W.to_csr(g.n, g.u, g.v, g.w))
    assert np.array_equal(cu, g.u) and np.array_equal(cv, g.v)
    assert np.array_equal(flags, want)


def test_sample_is_the_smallest_keys_off_the_forest(oracle_mod):
    rng = np.random.default_rng(8)
    n = 200
    u, v, w = _random_graph(rng, n, 900, lambda m: rng.uniform(1, 10, m))
    rp, col, ww = _csr(n, u, v, w)
    forest = oracle_mod.initial_sparsifier(n, rp, col, ww, 0, 1)
    for n_extra, seed in ((0, 1), (50, 2), (50, 3), (10_000, 4)):
        flags = oracle_mod.initial_sparsifier(n, rp, col, ww, n_extra, seed)
        assert np.all(flags[forest])
        extra = np.flatnonzero(flags & ~forest)
        off = np.flatnonzero(~forest)
        assert extra.size == min(n_extra, off.size)
        keys = sorted((oracle_mod.sample_key(seed, int(e)), int(e)) for e in off)
        assert set(extra.tolist()) == {e for _, e in keys[:n_extra]}


def test_sample_is_uniform(oracle_mod):
    """Each off-tree edge is picked with probability k / |off-tree|: chi-square
    of the pick counts over many seeds."""
    from scipy.stats import chisquare

    n = 60
    rng = np.random.default_rng(2)
    u, v, w = _random_graph(rng, n, 200, lambda m: rng.uniform(1, 10, m))
    rp, col, ww = _csr(n, u, v, w)
    forest = oracle_mod.initial_sparsifier(n, rp, col, ww, 0, 1)
    off = np.flatnonzero(~forest)
    k, seeds = 20, 3000
    counts = np.zeros(u.size)
    for seed in range(seeds):
        counts += oracle_mod.initial_sparsifier(n, rp, col, ww, k, seed) & ~forest
    expect = np.full(off.size, seeds * k / off.size)
    assert chisquare(counts[off], expect).pvalue > 1e-4


def test_degenerate_inputs(oracle_mod):
    # no edges at all
    flags = oracle_mod.initial_sparsifier(5, np.zeros(6, np.uint64), np.zeros(0, np.uint32),
                                          np.zeros(0), 3, 1)
    assert flags.size == 0
    # two components, each a triangle: forest of 4 edges; asking for more
    # off-tree edges than there are takes all
    u = np.array([0, 0, 1, 3, 3, 4], np.uint32)
    v = np.array([1, 2, 2, 4, 5, 5], np.uint32)
    w = np.array([1.0, 2.0, 3.0, 3.0, 2.0, 1.0])
    flags = oracle_mod.initial_sparsifier(6, *_csr(6, u, v, w), 0, 1)
    assert flags.tolist() == [False, True, True, True, True, False]
    assert oracle_mod.initial_sparsifier(6, *_csr(6, u, v, w), 99, 1).all()
