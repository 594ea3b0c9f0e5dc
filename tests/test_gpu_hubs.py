"""Long segments (more than 64 neighbours): prefix-sum selection in the walk,
prefix rebuilds after deletions and revivals, the workgroup-per-row merge and
relocation.  HIP library vs CPU oracle, element by element."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2505_02741_amd import workloads as W

from gpu_helpers import compare_batch, compare_state, make_pair, run_parity, say

pytestmark = pytest.mark.gpu

BATCHED = 4


@pytest.mark.parametrize("flags", [0, BATCHED])
def test_rmat_hubs_fully_dynamic(flags):
    wl = W.make_workload("rmat22", scale=13, batches=5, size_lo=200, size_hi=3000)
    deg = np.bincount(np.r_[wl.G.u, wl.G.v], minlength=wl.G.n)
    hdeg = np.bincount(np.r_[wl.hu, wl.hv], minlength=wl.G.n)
    say("rmat13: n", wl.G.n, "m", wl.G.m, "max deg G", int(deg.max()), "H", int(hdeg.max()),
        "rows > 64 in G:", int((deg > 64).sum()), "in H:", int((hdeg > 64).sum()))
    assert deg.max() > 64 and hdeg.max() > 64
    run_parity(wl, tag=f"rmat13 flags={flags}", flags=flags)


def _star_workload(n_leaves=300, seed=3):
    """A star (centre 0) plus a ring through the leaves, so walks can pass the
    centre in many ways."""
    rng = np.random.default_rng(seed)
    n = n_leaves + 1
    leaves = np.arange(1, n)
    u = np.r_[np.zeros(n_leaves, np.int64), leaves]
    v = np.r_[leaves, np.r_[leaves[1:], leaves[:1]]]
    cu, cv = W._canonical(n, u, v)
    w = rng.uniform(1.0, 10.0, cu.size)
    G = W.Graph(n, cu, cv, w)
    h = W.initial_sparsifier(G, rng)
    return W.Workload(name="star", G=G, h_mask=h, batches=[], seed_walk=77, s=64, L=12)


@pytest.mark.parametrize("flags,leaves", [(0, 300), (BATCHED, 300), (0, 6000), (BATCHED, 6000)])
def test_star_centre_deletions_revivals_and_bounce(flags, leaves):
    """With 6,000 leaves the centre's weight prefix is rebuilt in several
    chunks (after the deletions of phase 1 and after phase 4)."""
    wl = _star_workload(n_leaves=leaves)
    n = wl.G.n
    o, d = make_pair(wl, flags=flags, dead_end=1)
    z = np.zeros(0, np.uint32)
    try:
        # delete most spokes of the centre: tombstones in a long segment
        spokes = np.arange(1, 291, dtype=np.uint32)
        b1 = W.Batch(z, z, np.zeros(0), np.zeros(spokes.size, np.uint32), spokes)
        compare_batch(o, d, b1, tag="delete spokes")
        compare_state(o, d, "delete spokes")
        # walks through the centre now meet a long segment with one or few
        # live neighbours (dead ends, bounces) while leaves insert chords
        ins_u = np.arange(1, 120, dtype=np.uint32)
        ins_v = (ins_u + 150).astype(np.uint32)
        b2 = W.Batch(ins_u, ins_v, np.linspace(1, 9, ins_u.size), z, z)
        compare_batch(o, d, b2, tag="chords")
        # re-insert spokes (revive tombstones in the long segment)
        back = spokes[::3]
        b3 = W.Batch(np.zeros(back.size, np.uint32), back, np.linspace(2, 8, back.size), z, z)
        compare_batch(o, d, b3, tag="revive")
        compare_state(o, d, "revive")
    finally:
        d.close()
        o.close()


@pytest.mark.parametrize("flags", [0, BATCHED])
def test_wide_merge_more_than_one_chunk(flags):
    """One batch adds 2,500 neighbours to one vertex (three merge passes) and
    hundreds to a few others."""
    wl = W.make_workload("grid64", side=60, ins=0, batches=0, s=16, L=8)
    n = wl.G.n
    rng = np.random.default_rng(5)
    es = W.EdgeSet(wl.G)
    centre = 1830
    q = rng.choice(np.setdiff1d(np.arange(n), [centre]), 2600, replace=False)
    keep = ~es.contains(es.key(np.full(q.size, centre), q))
    q = q[keep][:2500]
    p = np.full(q.size, centre)
    others = rng.choice(n, 4, replace=False)
    extra_p, extra_q = [], []
    for c in others:
        qq = rng.choice(n, 300, replace=False)
        ok = (qq != c) & ~es.contains(es.key(np.full(qq.size, c), qq))
        extra_p.append(np.full(ok.sum(), c))
        extra_q.append(qq[ok])
    P = np.r_[p, np.concatenate(extra_p)]
    Q = np.r_[q, np.concatenate(extra_q)]
    k = es.key(P, Q)
    _, first = np.unique(k, return_index=True)
    sel = np.sort(first)
    P, Q = P[sel].astype(np.uint32), Q[sel].astype(np.uint32)
    say("  wide merge insertions:", P.size)
    z = np.zeros(0, np.uint32)
    b = W.Batch(P, Q, rng.uniform(1, 10, P.size), z, z)
    o, d = make_pair(wl, flags=flags)
    try:
        compare_batch(o, d, b, tag="wide merge")
        compare_state(o, d, "wide merge")
        # and walk through the new long segments
        z2 = W.make_workload("grid64", side=60, ins=200, batches=1, s=16, L=8)
        es.apply(es.key(P, Q), np.zeros(0, np.int64))
        pp, qq = W.local_insertions_lattice(es, 60, 2, 300, np.random.default_rng(8),
                                            np.zeros(0, np.int64))
        b2 = W.Batch(pp.astype(np.uint32), qq.astype(np.uint32), rng.uniform(1, 10, pp.size),
                     z, z)
        compare_batch(o, d, b2, tag="after wide merge")
        compare_state(o, d, "after wide merge")
        del z2
    finally:
        d.close()
        o.close()
