"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these re-types the oracle's own formulas: each compares it with an
independent source -- published known-answer vectors, numpy's Philox, dense
linear algebra, closed forms, brute-force enumeration of walk probabilities,
or an invariant stated in the paper.
"""
from __future__ import annotations

import math
import os
import subprocess
import sys
from collections import defaultdict, deque

import numpy as np
import pytest

from paper_2505_02741_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------
# helpers


def csr_of(n, u, v, w):
    return W.to_csr(n, np.asarray(u), np.asarray(v), np.asarray(w, dtype=np.float64))


def adjacency(n, u, v, w):
    adj = defaultdict(list)
    for a, b, x in zip(np.asarray(u).tolist(), np.asarray(v).tolist(), np.asarray(w).tolist()):
        adj[a].append((b, x))
        adj[b].append((a, x))
    for k in adj:
        adj[k].sort()
    return adj


def random_tree(n, rng):
    u = [int(rng.integers(0, i)) for i in range(1, n)]
    v = list(range(1, n))
    return np.array(u), np.array(v)


def tree_path(adj, p, q):
    par = {p: None}
    dq = deque([p])
    while dq:
        x = dq.popleft()
        for y, _ in adj[x]:
            if y not in par:
                par[y] = x
                dq.append(y)
    path = [q]
    while path[-1] != p:
        path.append(par[path[-1]])
    return path[::-1]


def connected(n, u, v, a, b):
    adj = defaultdict(list)
    for x, y in zip(u.tolist(), v.tolist()):
        adj[x].append(y)
        adj[y].append(x)
    seen = {a}
    dq = deque([a])
    while dq:
        x = dq.popleft()
        if x == b:
            return True
        for y in adj[x]:
            if y not in seen:
                seen.add(y)
                dq.append(y)
    return False


# --------------------------------------------------------------------------
# P7: Philox against the Random123 known-answer vectors and numpy


def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            rows.append((parts[0], int(parts[1]), [int(x, 16) for x in parts[2:]]))
    return rows


@pytest.mark.parametrize("row", _kat_rows(), ids=lambda r: r[0])
def test_philox_known_answers(oracle_mod, row):
    name, rounds, words = row
    assert rounds == 10
    ctr, key, exp = words[:4], words[4:6], words[6:10]
    fn = oracle_mod.philox4x32_10 if name == "philox4x32" else oracle_mod.philox4x64_10
    got = [int(x) for x in fn(ctr, key)]
    assert got == exp


def test_philox4x64_matches_numpy(oracle_mod):
    rng = np.random.default_rng(7)
    M = (1 << 64) - 1
    for _ in range(20):
        key = [int(x) for x in rng.integers(0, 2**63, 2, dtype=np.uint64)]
        ctr = [int(x) for x in rng.integers(0, 2**63, 4, dtype=np.uint64)]
        # numpy increments the counter before it draws a block: start one below
        v = sum(c << (64 * i) for i, c in enumerate(ctr)) - 1
        start = np.array([(v >> (64 * i)) & M for i in range(4)], dtype=np.uint64)
        bg = np.random.Philox(counter=start, key=np.array(key, dtype=np.uint64))
        expect = [int(x) for x in bg.random_raw(8)]
        got = [int(x) for x in oracle_mod.philox4x64_10(ctr, key)]
        ctr1 = list(ctr)
        ctr1[0] = (ctr1[0] + 1) & M
        got += [int(x) for x in oracle_mod.philox4x64_10(ctr1, key)]
        assert got == expect


def test_step_random_uses_counter_words(oracle_mod):
    """Step t of walker k of update uid reads block (t>>1, k, uid_lo, uid_hi)
    keyed by the seed; even steps take words 0-1, odd steps words 2-3.  Pinned
    through the first known-answer vector: seed 0, uid 0, walker 0 gives the
    all-zero counter."""
    kat = [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert oracle_mod.step_random(0, 0, 0, 0) == kat[0] | (kat[1] << 32)
    assert oracle_mod.step_random(0, 0, 0, 1) == kat[2] | (kat[3] << 32)
    pi = [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]
    # counter (0x243f6a88, 0x85a308d3, uid=(0x13198a2e, 0x03707344)), key pi
    seed = 0xA4093822 | (0x299F31D0 << 32)
    uid = 0x13198A2E | (0x03707344 << 32)
    t = 2 * 0x243F6A88 + 1
    assert oracle_mod.step_random(seed, uid, 0x85A308D3, t) == pi[2] | (pi[3] << 32)


# --------------------------------------------------------------------------
# P8: quantised weights


def test_quantize_special_values(oracle_mod):
    Q = 24
    assert oracle_mod.quantize(3.5, 3.5, Q) == 1 << Q
    assert oracle_mod.quantize(1.75, 3.5, Q) == 1 << (Q - 1)
    assert oracle_mod.quantize(1e-300, 3.5, Q) == 1  # clamped below
    assert oracle_mod.quantize(2.0**40, 1.0, Q) == 2**32 - 1  # clamped above
    # round half to even at exact .5: Q=1, w_ref=4 -> w/4*2 = w/2
    assert oracle_mod.quantize(5.0, 4.0, 1) == 2  # 2.5 -> 2
    assert oracle_mod.quantize(7.0, 4.0, 1) == 4  # 3.5 -> 4
    assert oracle_mod.quantize(3.0, 4.0, 1) == 2  # 1.5 -> 2
    # monotone in w
    ws = np.sort(np.random.default_rng(0).uniform(0.1, 10, 200))
    q = [oracle_mod.quantize(float(x), 10.0, Q) for x in ws]
    assert all(a <= b for a, b in zip(q, q[1:]))


# --------------------------------------------------------------------------
# P6: weight-biased choice excluding the previous vertex


def test_selection_frequencies_chi_square(oracle_mod):
    """prev -- x -- {a, b, c, d}: the walker starts at prev (a leaf), is forced
    to x, then picks among x's other neighbours with probability w/sum(w)."""
    ws = [1.0, 2.0, 3.5, 7.25]
    u = [0, 1, 1, 1, 1]
    v = [1, 2, 3, 4, 5]
    w = [5.0] + ws
    rp, col, ww = csr_of(6, u, v, w)
    counts = np.zeros(6)
    N = 0
    for uid in range(100):
        # target = the start vertex 0, which the walk can never re-enter
        r = oracle_mod.walk_csr(6, rp, col, ww, 0, 0, s=1000, L=2, uid=uid, seed=12345)
        ends = r["end"]
        assert np.all(r["steps"] == 2)
        counts += np.bincount(ends, minlength=6)
        N += ends.size
    expect = np.array([0, 0] + [N * x / sum(ws) for x in ws])
    chi2 = float(((counts[2:] - expect[2:]) ** 2 / expect[2:]).sum())
    assert counts[0] == 0 and counts[1] == 0
    assert chi2 < 25.0  # 3 dof; p ~ 1.5e-5


def test_selection_exact_with_coarse_quantisation(oracle_mod):
    """With Q=2 and w_ref=4 the quantised weights of w=1,2,3,4 are exactly the
    integers 1..4, so the choice probabilities are exactly qw/sum(qw) =
    0.1, 0.2, 0.3, 0.4; an off-by-one at a cumulative-sum boundary would move
    whole units of probability between neighbours."""
    ws = [1.0, 2.0, 3.0, 4.0]
    assert [oracle_mod.quantize(x, 4.0, 2) for x in ws] == [1, 2, 3, 4]
    u = [0, 1, 1, 1, 1]
    v = [1, 2, 3, 4, 5]
    rp, col, ww = csr_of(6, u, v, [2.0] + ws)
    counts = np.zeros(6)
    N = 0
    for uid in range(60):
        r = oracle_mod.walk_csr(6, rp, col, ww, 0, 0, s=1000, L=2, uid=uid, seed=77, Q=2,
                                w_ref=4.0)
        counts += np.bincount(r["end"], minlength=6)
        N += 1000
    p = np.array([0.1, 0.2, 0.3, 0.4])
    emp = counts[2:] / N
    assert np.all(np.abs(emp - p) < 5 * np.sqrt(p * (1 - p) / N))


def _exact_outcomes(adj, p, q, L, K=None, w_pq=None, bounce=False):
    """Exact distribution of (hit, steps, end) of one walker by enumeration of
    every non-backtracking trajectory, with real-valued weights."""
    out = defaultdict(float)

    def rec(x, prev, t, prob, R):
        if t == L:
            out[(0, t, x)] += prob
            return
        cands = [(c, wc) for c, wc in adj[x] if c != prev]
        if not cands:
            if bounce and prev is not None:
                cands = [(c, wc) for c, wc in adj[x] if c == prev]
            else:
                out[(0, t, x)] += prob
                return
        tot = sum(wc for _, wc in cands)
        for c, wc in cands:
            pr = prob * wc / tot
            R2 = R + 1.0 / wc
            if K is not None and w_pq * R2 > K:
                out[(0, t + 1, c)] += pr
            elif c == q:
                out[(1, t + 1, c)] += pr
            else:
                rec(c, x, t + 1, pr, R2)

    rec(p, None, 0, 1.0, 0.0)
    return out


@pytest.mark.parametrize("bounce", [False, True])
def test_walk_distribution_matches_enumeration(oracle_mod, bounce):
    # a small graph with cycles, a pendant path and a leaf
    u = [0, 0, 1, 1, 2, 3, 4, 5, 6]
    v = [1, 2, 2, 3, 3, 4, 5, 6, 7]
    w = [1.0, 3.0, 2.0, 0.5, 4.0, 1.5, 2.5, 1.0, 6.0]
    n = 8
    p, q, L = 0, 5, 7
    adj = adjacency(n, u, v, w)
    exact = _exact_outcomes(adj, p, q, L, bounce=bounce)
    assert abs(sum(exact.values()) - 1.0) < 1e-12
    rp, col, ww = csr_of(n, u, v, w)
    counts = defaultdict(int)
    N = 0
    for uid in range(150):
        r = oracle_mod.walk_csr(n, rp, col, ww, p, q, s=1000, L=L, uid=uid, seed=99,
                                bounce=bounce)
        for h, st, e in zip(r["hit"].tolist(), r["steps"].tolist(), r["end"].tolist()):
            counts[(int(h), st, e)] += 1
        N += 1000
    assert set(counts) <= set(exact)
    for key, pr in exact.items():
        emp = counts.get(key, 0) / N
        sd = math.sqrt(max(pr * (1 - pr), 1e-12) / N)
        assert abs(emp - pr) < 5 * sd + 1e-9, (key, emp, pr)


def test_walk_distribution_with_threshold(oracle_mod):
    u = [0, 0, 1, 1, 2, 3, 4]
    v = [1, 2, 2, 3, 3, 4, 0]
    w = [1.0, 3.0, 2.0, 0.5, 4.0, 1.5, 2.0]
    n, p, q, L = 5, 0, 3, 9
    K, w_pq = 2.2, 1.7
    adj = adjacency(n, u, v, w)
    exact = _exact_outcomes(adj, p, q, L, K=K, w_pq=w_pq)
    rp, col, ww = csr_of(n, u, v, w)
    counts = defaultdict(int)
    N = 0
    for uid in range(120):
        r = oracle_mod.walk_csr(n, rp, col, ww, p, q, s=1000, L=L, uid=uid, seed=5,
                                use_K=True, K=K, w_pq=w_pq)
        for h, st, e in zip(r["hit"].tolist(), r["steps"].tolist(), r["end"].tolist()):
            counts[(int(h), st, e)] += 1
        N += 1000
    assert set(counts) <= set(exact)
    for key, pr in exact.items():
        emp = counts.get(key, 0) / N
        sd = math.sqrt(max(pr * (1 - pr), 1e-12) / N)
        assert abs(emp - pr) < 5 * sd + 1e-9, (key, emp, pr)


# --------------------------------------------------------------------------
# P1 / P2: resistance of the walk against the exact effective resistance


def test_tree_walk_is_unique_path_and_exact_resistance(oracle_mod):
    from oracle import spectral

    rng = np.random.default_rng(3)
    for trial in range(6):
        n = 30
        u, v = random_tree(n, rng)
        w = rng.uniform(0.2, 5.0, n - 1)
        adj = adjacency(n, u, v, w)
        Lm = spectral.laplacian(n, u, v, w)
        p, q = (int(x) for x in rng.choice(n, 2, replace=False))
        reff = spectral.effective_resistance(Lm, p, q)
        path = tree_path(adj, p, q)
        rp, col, ww = csr_of(n, u, v, w)
        r = oracle_mod.walk_csr(n, rp, col, ww, p, q, s=1024, L=n, uid=trial, seed=11)
        assert r["hit"].any()
        for k in np.flatnonzero(r["hit"]):
            st = int(r["steps"][k])
            assert r["traj"][k, : st + 1].tolist() == path
            assert abs(r["R"][k] - reff) <= 1e-12 * reff


def test_hit_resistance_upper_bounds_effective_resistance(oracle_mod):
    from oracle import spectral

    rng = np.random.default_rng(4)
    n, u, v = W.grid2d(6)
    w = rng.uniform(0.5, 4.0, u.size)
    Lm = spectral.laplacian(n, u, v, w)
    rp, col, ww = csr_of(n, u, v, w)
    nhits = 0
    for trial in range(8):
        p, q = (int(x) for x in rng.choice(n, 2, replace=False))
        reff = spectral.effective_resistance(Lm, p, q)
        r = oracle_mod.walk_csr(n, rp, col, ww, p, q, s=512, L=24, uid=trial, seed=1)
        hits = r["R"][r["hit"]]
        nhits += hits.size
        assert np.all(hits >= reff * (1 - 1e-12))
    assert nhits > 100


# --------------------------------------------------------------------------
# P3: path graph closed form


def test_path_graph_closed_form(oracle_mod):
    n = 10
    u = np.arange(n - 1)
    v = u + 1
    w = np.array([1.0, 2.0, 0.5, 3.0, 1.5, 2.5, 4.0, 0.25, 1.0])
    rp, col, ww = csr_of(n, u, v, w)
    p, q = 3, 7
    r_fwd = 0.0
    for i in range(3, 7):
        r_fwd = r_fwd + 1.0 / w[i]
    r_back = 0.0
    for i in (2, 1, 0):
        r_back = r_back + 1.0 / w[i]
    res = oracle_mod.walk_csr(n, rp, col, ww, p, q, s=1000, L=32, seed=8)
    fwd = res["hit"]
    # forward walkers hit at step 4 with the path resistance, backward ones
    # stop at the leaf 0 after 3 steps
    assert np.all(res["steps"][fwd] == 4) and np.all(res["R"][fwd] == r_fwd)
    assert np.all(res["steps"][~fwd] == 3) and np.all(res["end"][~fwd] == 0)
    assert np.all(res["R"][~fwd] == r_back)
    frac = fwd.mean()
    pf = w[3] / (w[2] + w[3])
    assert abs(frac - pf) < 5 * math.sqrt(pf * (1 - pf) / 1000)
    # the step limit below the hop distance removes every hit
    short = oracle_mod.walk_csr(n, rp, col, ww, p, q, s=1000, L=3, seed=8)
    assert not short["hit"].any()
    # threshold: hit iff w_pq * R <= K
    for K in (r_fwd * 2.0 - 1e-9, r_fwd * 2.0, r_fwd * 2.0 + 1e-9):
        rk = oracle_mod.walk_csr(n, rp, col, ww, p, q, s=1000, L=32, seed=8, use_K=True,
                                 K=K, w_pq=2.0)
        assert rk["hit"].any() == (2.0 * r_fwd <= K)
    # bounce at the leaf: backward walkers return and hit after 3+1+6 steps
    rb = oracle_mod.walk_csr(n, rp, col, ww, p, q, s=1000, L=32, seed=8, bounce=True)
    assert rb["hit"].all()
    back = ~fwd
    assert np.all(rb["steps"][back] == 10)
    exp = 0.0
    for i in (2, 1, 0, 0, 1, 2, 3, 4, 5, 6):
        exp = exp + 1.0 / w[i]
    assert np.all(rb["R"][back] == exp)


# --------------------------------------------------------------------------
# P4: unit weights, w_pq = 1: threshold K = k equals a k-step limit
# (the case study of Sec. III-E equates K = 4 with a limit of four steps)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6])
def test_threshold_equals_step_limit_for_unit_weights(oracle_mod, k):
    n, u, v = W.grid2d(7)
    w = np.ones(u.size)
    rp, col, ww = csr_of(n, u, v, w)
    L = 12
    rng = np.random.default_rng(k)
    for trial in range(5):
        p, q = (int(x) for x in rng.choice(n, 2, replace=False))
        a = oracle_mod.walk_csr(n, rp, col, ww, p, q, s=256, L=L, uid=trial, seed=2,
                                use_K=True, K=float(k), w_pq=1.0)
        b = oracle_mod.walk_csr(n, rp, col, ww, p, q, s=256, L=min(L, k), uid=trial, seed=2)
        assert np.array_equal(a["hit"], b["hit"])
        h = a["hit"]
        assert np.array_equal(a["steps"][h], b["steps"][h])
        assert np.array_equal(a["R"][h], b["R"][h])
        assert np.all(a["steps"][~h & (a["steps"] > k)] == k + 1)


# --------------------------------------------------------------------------
# P5: non-backtracking and dead ends


@pytest.mark.parametrize("bounce", [False, True])
def test_non_backtracking_and_dead_ends(oracle_mod, bounce):
    rng = np.random.default_rng(21)
    n = 60
    tu, tv = random_tree(n, rng)
    extra = rng.choice(n, (8, 2))
    u = np.concatenate([tu, extra[:, 0]])
    v = np.concatenate([tv, extra[:, 1]])
    nn, u, v = n, *W._canonical(n, u, v)
    w = rng.uniform(0.5, 3.0, u.size)
    adj = adjacency(n, u, v, w)
    deg = {x: len(adj[x]) for x in range(n)}
    rp, col, ww = csr_of(n, u, v, w)
    L = 20
    for trial in range(10):
        p, q = (int(x) for x in rng.choice(n, 2, replace=False))
        r = oracle_mod.walk_csr(n, rp, col, ww, p, q, s=200, L=L, uid=trial, seed=3,
                                bounce=bounce)
        for k in range(200):
            st = int(r["steps"][k])
            tr = r["traj"][k, : st + 1].tolist()
            for t in range(1, st):
                back = tr[t + 1] == tr[t - 1]
                if back:
                    # only a forced bounce at a vertex whose sole neighbour is prev
                    assert bounce and deg[tr[t]] == 1
            if not r["hit"][k] and st < L:
                # stopped early without a hit: a dead end (TERMINATE policy)
                assert not bounce or st == 0
                x = tr[-1]
                assert deg[x] == 0 or (deg[x] == 1 and st > 0)
            assert r["end"][k] == tr[-1]


# --------------------------------------------------------------------------
# P9: the dense spectral tooling (kappa, Eq. 5, Eqs. 9-11)


def test_spectral_tooling_pins():
    from oracle import spectral

    rng = np.random.default_rng(5)
    n, u, v = W.grid2d(5)
    w = rng.uniform(0.5, 3.0, u.size)
    LG = spectral.laplacian(n, u, v, w)
    assert abs(spectral.relative_condition_number(LG, LG) - 1.0) < 1e-9
    # unit cycle vs the path left after removing one edge: kappa = n
    for m in (5, 9, 16):
        cu = np.arange(m)
        cv = (cu + 1) % m
        LC = spectral.laplacian(m, cu, cv, np.ones(m))
        LP = spectral.laplacian(m, cu[:-1], cv[:-1], np.ones(m - 1))
        assert abs(spectral.relative_condition_number(LC, LP) - m) < 1e-8 * m
    # a spanning tree plus a few edges, with a leaf of G whose edge is kept:
    # lambda_min(L_G, L_H) = 1 (Eqs. 9-10) and w_e R_H(e) <= kappa (Eq. 11)
    G = W.Graph(n, u, v, w)
    mask = W.max_spanning_forest(n, u, v, w)
    lu = np.append(u, n)  # add a pendant vertex n, attached to vertex 0
    lv = np.append(v, 0)
    lw = np.append(w, 2.0)
    lm = np.append(mask, True)
    LG2 = spectral.laplacian(n + 1, lu, lv, lw)
    LH2 = spectral.laplacian(n + 1, lu[lm], lv[lm], lw[lm])
    lam = spectral.generalized_eigs(LG2, LH2)
    assert abs(lam[0] - 1.0) < 1e-9
    kappa = lam[-1] / lam[0]
    for a, b, x in zip(lu, lv, lw):
        assert x * spectral.effective_resistance(LH2, int(a), int(b)) <= kappa * (1 + 1e-9)
    # Eq. 5 with every eigenpair: Delta_N = w b^T L_H^+ b
    LH = spectral.laplacian(n, u[mask], v[mask], w[mask])
    p, q = 0, n - 1
    d = spectral.spectral_distortion(LH, p, q, 1.7)
    assert abs(d - 1.7 * spectral.effective_resistance(LH, p, q)) < 1e-9 * d
    del G


# --------------------------------------------------------------------------
# P10 / P11: batch semantics on seeded workloads


def _oracle_for(oracle_mod, wl, **kw):
    rp, col, w = W.to_csr(wl.G.n, wl.G.u, wl.G.v, wl.G.w)
    return oracle_mod.Oracle(wl.G.n, rp, col, w, wl.hu, wl.hv, seed=wl.seed_walk, s=wl.s,
                             L=wl.L, K=wl.K, **kw)


def _edge_dict(u, v, w):
    return {(int(a), int(b)): float(x) for a, b, x in zip(u, v, w)}


@pytest.mark.parametrize("name,over", [("grid64", {}),
                                       ("mesh128", dict(side=9, ins=60, dels=60, batches=6))])
def test_batch_invariants(oracle_mod, name, over):
    wl = W.make_workload(name, **over)
    o = _oracle_for(oracle_mod, wl)
    G = _edge_dict(*o.query("G"))
    H = _edge_dict(*o.query("H"))
    for b in wl.batches:
        r = o.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, record_walkers=True)
        ni = b.n_ins
        dkeys = {(min(a, c), max(a, c)) for a, c in zip(b.du.tolist(), b.dv.tolist())}
        # in_H flags are membership tests of H_t
        for j, key in enumerate(zip(b.du.tolist(), b.dv.tolist())):
            assert r["flag"][ni + j] == ((min(key), max(key)) in H)
        # accepted <=> no walker reached q
        assert np.array_equal(r["flag"][:ni], 1 - r["any_hit"][:ni])
        # per-update minimum and winner agree with the per-walker records
        wk = r["walkers"]
        for i in range(b.size):
            sl = slice(i * wl.s, (i + 1) * wl.s)
            hits = np.flatnonzero(wk["hit"][sl])
            assert r["any_hit"][i] == (hits.size > 0)
            assert r["steps"][i] == wk["steps"][sl].astype(np.int64).sum()
            if hits.size:
                R = wk["R"][sl][hits]
                assert r["Rmin"][i] == R.min()
                if i >= ni:
                    assert r["winner"][i] == hits[np.argmin(R)]
            else:
                assert math.isinf(r["Rmin"][i])
        Gn = _edge_dict(*o.query("G"))
        Hn = _edge_dict(*o.query("H"))
        # G_{t+1} = G_t + I - D exactly, with the inserted weights
        expect = dict(G)
        for key in dkeys:
            del expect[key]
        for a, c, x in zip(b.iu.tolist(), b.iv.tolist(), b.iw.tolist()):
            expect[(min(a, c), max(a, c))] = x
        assert Gn == expect
        # H subset of G with equal weights; H_{t+1} contains H_t - D
        for key, x in Hn.items():
            assert Gn[key] == x
        for key in H:
            if key not in dkeys:
                assert key in Hn
        # accepted insertions are exactly the new H edges that are insertions
        ins_keys = [(min(a, c), max(a, c)) for a, c in zip(b.iu.tolist(), b.iv.tolist())]
        for i, key in enumerate(ins_keys):
            assert (key in Hn) == bool(r["flag"][i])
        # P11: a deletion walk that hit leaves u and v connected in H_{t+1}
        hu_, hv_, _ = o.query("H")
        for j in range(b.n_del):
            if r["flag"][ni + j] and r["any_hit"][ni + j]:
                assert connected(wl.G.n, hu_, hv_, int(b.du[j]), int(b.dv[j]))
            if r["flag"][ni + j] and not r["any_hit"][ni + j]:
                assert r["n_rec"][ni + j] <= 2
        G, H = Gn, Hn
    assert o.uid_base == sum(b.size for b in wl.batches)


def test_rebuild_invariance(oracle_mod):
    """Re-creating the state from (G_t, H_t, uid_base) reproduces every later
    result: the state is exactly the two edge sets and the update counter."""
    wl = W.make_workload("mesh128", side=8, ins=40, dels=40, batches=4)
    a = _oracle_for(oracle_mod, wl)
    for b in wl.batches[:2]:
        a.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv)
    gu, gv, gw = a.query("G")
    hu, hv, _ = a.query("H")
    rp, col, w = W.to_csr(wl.G.n, gu, gv, gw)
    b_ = oracle_mod.Oracle(wl.G.n, rp, col, w, hu, hv, seed=wl.seed_walk, s=wl.s, L=wl.L,
                           w_ref=a.w_ref, uid_base=a.uid_base)
    for b in wl.batches[2:]:
        ra = a.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, record_walkers=True)
        rb = b_.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, record_walkers=True)
        for k in ("flag", "any_hit", "winner", "n_rec", "steps", "Rmin"):
            assert np.array_equal(ra[k], rb[k])
        for k in ("hit", "steps", "end", "R"):
            assert np.array_equal(ra["walkers"][k], rb["walkers"][k])
    assert _edge_dict(*a.query("H")) == _edge_dict(*b_.query("H"))


def test_thread_count_invariance():
    """Phase 2 reads only the batch snapshot: results do not depend on how
    many threads run it."""
    code = r"""
import sys, numpy as np
sys.path.insert(0, %r)
import oracle
from paper_2505_02741_amd import workloads as W
wl = W.make_workload("mesh128", side=8, ins=50, dels=50, batches=3)
rp, col, w = W.to_csr(wl.G.n, wl.G.u, wl.G.v, wl.G.w)
o = oracle.Oracle(wl.G.n, rp, col, w, wl.hu, wl.hv, seed=wl.seed_walk, s=wl.s, L=wl.L)
acc = []
for b in wl.batches:
    r = o.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, record_walkers=True)
    acc.append(r["walkers"]["R"].sum() + r["flag"].sum())
u, v, ww = o.query("H")
print(repr((float(np.sum(acc)), int(u.size), float(ww.sum()))))
""" % os.path.dirname(HERE)
    outs = []
    for th in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=th)
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, check=True,
                                   capture_output=True, text=True).stdout)
    assert outs[0] == outs[1]


# --------------------------------------------------------------------------
# validation


def test_validation_errors(oracle_mod):
    wl = W.make_workload("grid64", side=8, ins=5, batches=1)
    o = _oracle_for(oracle_mod, wl)
    gu, gv, _ = o.query("G")
    e0 = (int(gu[0]), int(gv[0]))
    z = np.zeros(0)
    cases = [
        (dict(iu=[0], iv=[0], iw=[1.0]), "SELF_LOOP"),
        (dict(iu=[0], iv=[64], iw=[1.0]), "VERTEX_RANGE"),
        (dict(iu=[0], iv=[9], iw=[0.0]), "BAD_WEIGHT"),
        (dict(iu=[0], iv=[9], iw=[math.inf]), "BAD_WEIGHT"),
        (dict(iu=[e0[0]], iv=[e0[1]], iw=[1.0]), "EDGE_EXISTS"),
        (dict(iu=[0, 9], iv=[9, 0], iw=[1.0, 2.0]), "DUPLICATE_IN_BATCH"),
        (dict(du=[0], dv=[9]), "EDGE_MISSING"),
        (dict(du=[e0[0], e0[1]], dv=[e0[1], e0[0]]), "DUPLICATE_IN_BATCH"),
        # precedence: the first bad insertion wins over a later bad deletion
        (dict(iu=[0, 0], iv=[9, 0], iw=[1.0, 1.0], du=[0], dv=[9]), "SELF_LOOP"),
    ]
    before = _edge_dict(*o.query("H"))
    uid = o.uid_base
    for kw, name in cases:
        args = dict(iu=z, iv=z, iw=z, du=z, dv=z)
        args.update(kw)
        with pytest.raises(oracle_mod.OracleError) as ei:
            o.apply_batch(**args)
        assert ei.value.name == name
    # failed calls change nothing
    assert _edge_dict(*o.query("H")) == before and o.uid_base == uid
    with pytest.raises(oracle_mod.OracleError) as ei:
        o.apply_batch([0], [9], [1.0], z, z, s=[2000])
    assert ei.value.name == "INVALID_ARG"
