"""dyg_initial_sparsifier (maximum spanning forest by Boruvka rounds on the
GPU + the keyed off-tree sample) against the oracle's Kruskal and sample,
edge for edge, on grid, mesh and R-MAT inputs and on degenerate ones."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2505_02741_amd import workloads as W

from gpu_helpers import say

pytestmark = pytest.mark.gpu


def _both(n, rp, col, w, n_extra, seed):
    import oracle
    from paper_2505_02741_amd import dygrass as D

    flags = oracle.initial_sparsifier(n, rp, col, w, n_extra, seed)
    cu, cv, _ = oracle.canonical_edges(n, rp, col, w)
    hu, hv = D.dyg_initial_sparsifier(n, rp, col, w, n_extra, seed)
    return (cu[flags], cv[flags]), (hu, hv)


@pytest.mark.parametrize("name,over,frac", [
    ("grid1024", dict(side=256), 0.1),
    ("mesh128", dict(side=32), 0.1),
    ("rmat22", dict(scale=16), 0.1),
    ("grid64", dict(side=64), 0.0),
    ("rmat22", dict(scale=12), 100.0),  # more than every off-tree edge: all of them
])
def test_initial_sparsifier_equals_oracle(name, over, frac):
    wl = W.make_workload(name, batches=0, **over)
    g = wl.G
    rp, col, w = W.to_csr(g.n, g.u, g.v, g.w)
    n_extra = int(round(frac * g.n))
    (ou, ov), (hu, hv) = _both(g.n, rp, col, w, n_extra, seed=12345)
    say(f"  {name} {over}: n={g.n} m={g.m} H0={ou.size} (n_extra {n_extra})")
    assert np.array_equal(hu, ou) and np.array_equal(hv, ov)


def test_initial_sparsifier_full_grid1024():
    """The 1024x1024 grid at its real size (2.1M edges, lognormal weights)."""
    wl = W.make_workload("grid1024", batches=0)
    g = wl.G
    rp, col, w = W.to_csr(g.n, g.u, g.v, g.w)
    (ou, ov), (hu, hv) = _both(g.n, rp, col, w, int(round(0.1 * g.n)), seed=7)
    assert np.array_equal(hu, ou) and np.array_equal(hv, ov)
    assert ou.size == g.n - 1 + int(round(0.1 * g.n))


def test_initial_sparsifier_degenerate():
    from paper_2505_02741_amd import dygrass as D

    # no edges at all
    hu, hv = D.dyg_initial_sparsifier(4, np.zeros(5, np.uint64), np.zeros(0, np.uint32),
                                      np.zeros(0), 3, 1)
    assert hu.size == 0
    # two triangles with tied weights, forest only and everything
    u = np.array([0, 0, 1, 3, 3, 4], np.uint32)
    v = np.array([1, 2, 2, 4, 5, 5], np.uint32)
    w = np.array([2.0, 2.0, 2.0, 1.0, 1.0, 1.0])
    rp, col, ww = W.to_csr(6, u, v, w)
    for n_extra in (0, 1, 2, 9):
        (ou, ov), (hu, hv) = _both(6, rp, col, ww, n_extra, seed=3)
        assert np.array_equal(hu, ou) and np.array_equal(hv, ov), n_extra
    # a star: every edge is in the forest
    n = 1000
    u = np.zeros(n - 1, np.uint32)
    v = np.arange(1, n, dtype=np.uint32)
    rp, col, ww = W.to_csr(n, u, v, np.linspace(1.0, 2.0, n - 1))
    hu, hv = D.dyg_initial_sparsifier(n, rp, col, ww, 50, 1)
    assert hu.size == n - 1
    # invalid input is refused before the GPU is used
    with pytest.raises(D.DygError):
        D.dyg_initial_sparsifier(3, np.array([0, 1, 1, 1], np.uint64), np.array([0], np.uint32),
                                 np.array([1.0]), 0, 1)
