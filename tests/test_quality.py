"""The mid-scale quality harness (oracle/quality.py): the sparse relative
condition number pinned to the dense one and to closed forms, and the trend
of the paper's Tables II and III on a synthetic insertion stream."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2505_02741_amd import workloads as W


def test_sparse_kappa_matches_dense():
    from oracle import quality as Q
    from oracle import spectral

    # grids, and a mesh whose face diagonals make it non-bipartite
    for seed, gen, side, extra in ((1, W.grid2d, 6, 0.1), (2, W.grid2d, 8, 0.3),
                                   (3, W.grid2d, 9, 0.0), (4, W.mesh3d, 4, 0.2)):
        rng = np.random.default_rng(seed)
        n, u, v = gen(side)
        w = rng.lognormal(0.0, 1.0, u.size)
        hm = W.max_spanning_forest(n, u, v, w) | (rng.random(u.size) < extra)
        dense = spectral.relative_condition_number(spectral.laplacian(n, u, v, w),
                                                   spectral.laplacian(n, u[hm], v[hm], w[hm]))
        sparse = Q.relative_condition_number(n, (u, v, w), (u[hm], v[hm], w[hm]))
        assert abs(sparse - dense) <= 1e-8 * dense, (seed, sparse, dense)


def test_kappa_closed_forms():
    from oracle import quality as Q

    # unit cycle against the path left after removing one edge: kappa = m
    for m in (50, 400):
        cu = np.arange(m)
        cv = (cu + 1) % m
        k = Q.relative_condition_number(m, (cu, cv, np.ones(m)), (cu[:-1], cv[:-1], np.ones(m - 1)))
        assert abs(k - m) < 1e-6 * m
    # a graph against itself, and against itself with weights scaled by c:
    # every generalized eigenvalue is 1 (resp. 1/c)
    rng = np.random.default_rng(4)
    n, u, v = W.grid2d(30)
    w = rng.uniform(0.5, 2.0, u.size)
    lo, hi = Q.pencil_extremes(n, (u, v, w), (u, v, w))
    assert abs(lo - 1.0) < 1e-8 and abs(hi - 1.0) < 1e-8
    lo, hi = Q.pencil_extremes(n, (u, v, w), (u, v, 4.0 * w))
    assert abs(lo - 0.25) < 1e-8 and abs(hi - 0.25) < 1e-8
    # a subgraph H of G with a pendant vertex of G kept in H: lambda_min = 1
    # (Eqs. 9-10), lambda_max >= 1
    hm = W.max_spanning_forest(n, u, v, w)
    lu, lv, lw = np.append(u, n), np.append(v, 0), np.append(w, 1.5)
    lm = np.append(hm, True)
    lo, hi = Q.pencil_extremes(n + 1, (lu, lv, lw), (lu[lm], lv[lm], lw[lm]))
    assert abs(lo - 1.0) < 1e-8 and hi > 1.0


def test_pcg_solves_and_exact_preconditioner_takes_one_step():
    import scipy.sparse.linalg as sla

    from oracle import quality as Q

    rng = np.random.default_rng(6)
    n, u, v = W.grid2d(20)
    w = rng.lognormal(0.0, 1.0, u.size)
    hm = W.max_spanning_forest(n, u, v, w) | (rng.random(u.size) < 0.1)
    b = rng.standard_normal(n - 1)
    # preconditioned by G itself: one step
    it, x = Q.pcg_iterations(n, (u, v, w), (u, v, w), b=b)
    assert it == 1
    # by a sparsifier: more steps, and x solves the grounded system
    it, x = Q.pcg_iterations(n, (u, v, w), (u[hm], v[hm], w[hm]), b=b)
    A = Q.grounded_laplacian(n, u, v, w)
    assert it > 1
    assert np.linalg.norm(A @ x - b) <= 1e-8 * np.linalg.norm(b)
    xd = sla.splu(A).solve(b)
    assert np.linalg.norm(x - xd) <= 1e-6 * np.linalg.norm(xd)


def test_off_tree_density():
    from oracle import quality as Q

    assert Q.off_tree_density(100, 99) == pytest.approx(-0.01)  # a spanning tree
    assert Q.off_tree_density(100, 110) == pytest.approx(0.1)


@pytest.mark.parametrize("name,seed,over", [
    ("grid1024", 1, dict(side=32, ins=25, batches=10)),
    ("grid1024", 2, dict(side=32, ins=25, batches=10)),
    ("mesh128", 1, dict(side=10, ins=25, dels=0, batches=10)),
], ids=["grid32-s1", "grid32-s2", "mesh10-s1"])
def test_stream_trend_of_tables_two_to_four(name, seed, over):
    """Ten insertion batches adding 25% of |V| edges to a 32x32 lognormal grid
    or a 10^3 FEM-like mesh (the stream shape of Sec. IV): with H left alone
    kappa and the PCG
    iteration count grow; adding every edge gives the densest H; the oracle's
    updates (K = kappa of the initial pair) keep H far sparser than that
    while kappa stays at or below its initial value and PCG needs fewer
    iterations than with H left alone (Tables II-IV)."""
    from oracle import quality as Q

    wl = W.make_workload(name, seed=seed, **over)
    r = Q.stream_trend(wl)
    d0, k0, i0 = r["initial"]
    assert r["K"] == pytest.approx(k0)
    d_none, k_none, i_none = r["no_update"]
    d_all, k_all, i_all = r["no_filter"]
    d_dyg, k_dyg, i_dyg = r["dygrass"]
    assert d_none == pytest.approx(d0) and k_none > k0 and i_none > i0
    assert i_all < i_dyg < i_none
    assert d_all > d_dyg > d0
    assert k_dyg <= k0 and k_dyg < k_none
    # H with every edge contains the oracle's H, so lambda_max can only be
    # lower; lambda_min is 1 for both (a vertex whose edges all lie in H)
    assert k_all <= k_dyg
    # one update per batch (each sees the previous ones): the same picture
    d_seq, k_seq, i_seq = r["sequential"]
    assert d_all > d_seq > d0 and k_seq < k_none and i_seq < i_none


def test_unweighted_selection_through_a_huge_reference_weight():
    """A reference weight of 10^300 quantises every weight to the clamp
    floor 1, so the walkers choose uniformly (resistance still uses 1/w);
    the update rule still keeps H sparse and kappa below H left alone."""
    import oracle
    from oracle import quality as Q

    for w in (1e-3, 0.5, 1.0, 7.0, 1e6):
        assert oracle.quantize(w, 1e300) == 1
    wl = W.make_workload("grid1024", seed=1, side=32, ins=25, batches=10)
    r = Q.stream_trend(wl, w_ref=1e300)
    d0, k0, _ = r["initial"]
    d_dyg, k_dyg, _ = r["dygrass"]
    assert r["no_filter"][0] > d_dyg > d0
    assert k_dyg < r["no_update"][1]


def test_pins_reject_planted_mistakes(monkeypatch):
    """Plausible mistakes in the grounded Laplacian (a dropped diagonal term,
    a flipped off-diagonal sign, a row grounded without its column) change
    the sparse kappa away from the dense one, which the first pin checks.
    The graph has triangles: on a bipartite graph D + A = S (D - A) S for a
    diagonal sign matrix S, so a flipped sign would leave kappa unchanged."""
    import scipy.sparse as sp

    from oracle import quality as Q
    from oracle import spectral

    rng = np.random.default_rng(2)
    n, u, v = W.mesh3d(4)
    w = rng.lognormal(0.0, 1.0, u.size)
    hm = W.max_spanning_forest(n, u, v, w) | (rng.random(u.size) < 0.3)
    dense = spectral.relative_condition_number(spectral.laplacian(n, u, v, w),
                                               spectral.laplacian(n, u[hm], v[hm], w[hm]))
    good = Q.grounded_laplacian

    def no_v_diagonal(n_, u_, v_, w_, root=0):
        u_, v_, w_ = (np.asarray(x) for x in (u_, v_, w_))
        Lm = sp.coo_matrix((np.concatenate([-w_, -w_, w_]),
                            (np.concatenate([u_, v_, u_]), np.concatenate([v_, u_, u_]))),
                           shape=(n_, n_)).tocsr()
        keep = np.arange(1, n_)
        return Lm[keep][:, keep].tocsc()

    def flipped_sign(n_, u_, v_, w_, root=0):
        L = good(n_, u_, v_, w_, root)
        d = sp.diags(L.diagonal())
        return (2 * d - L).tocsc()

    def row_only(n_, u_, v_, w_, root=0):
        u_, v_, w_ = (np.asarray(x) for x in (u_, v_, w_))
        Lm = sp.coo_matrix((np.concatenate([-w_, -w_, w_, w_]),
                            (np.concatenate([u_, v_, u_, v_]), np.concatenate([v_, u_, u_, v_]))),
                           shape=(n_, n_)).tocsr()
        return (Lm[1:][:, :-1]).tocsc()

    for bad in (no_v_diagonal, flipped_sign, row_only):
        monkeypatch.setattr(Q, "grounded_laplacian", bad)
        try:
            k = Q.relative_condition_number(n, (u, v, w), (u[hm], v[hm], w[hm]))
        except Exception:
            continue  # failing outright is rejection too
        finally:
            monkeypatch.setattr(Q, "grounded_laplacian", good)
        assert abs(k - dense) > 1e-6 * dense, bad.__name__
