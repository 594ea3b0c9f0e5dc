"""Pins of the oracle's variants of the update rule (the alternatives the
paper names or leaves open), each on a hand-built graph whose answer follows
from its structure:

* BOTH_ENDS: odd walkers start at the second endpoint and aim at the first
  (Sec. III-C lets the walkers start at either endpoint);
* LOOP_ERASED: a hitting deletion recovers the chronological loop erasure of
  the winner's path (Sec. III-C recovers the edges along the path; erasing
  its loops is the alternative);
* TWO_STAGE: deletions and their recoveries enter H before the insertion
  walks (Sec. III-F defers every update to the batch end; this variant
  repairs H first).
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_2505_02741_amd import workloads as W


def _oracle(oracle_mod, n, edges, h_edges, *, variant=0, s=8, L=16, seed=11):
    u = np.array([a for a, _, _ in edges], dtype=np.uint32)
    v = np.array([b for _, b, _ in edges], dtype=np.uint32)
    w = np.array([x for _, _, x in edges], dtype=np.float64)
    rp, col, ww = W.to_csr(n, u, v, w)
    hu = np.array([a for a, _ in h_edges], dtype=np.uint32)
    hv = np.array([b for _, b in h_edges], dtype=np.uint32)
    return oracle_mod.Oracle(n, rp, col, ww, hu, hv, seed=seed, s=s, L=L, variant=variant)


def _H(o):
    u, v, _ = o.query("H")
    return {(int(a), int(b)) for a, b in zip(u, v)}


Z = np.zeros(0, np.uint32)
ZW = np.zeros(0)

# u=0 -- a=1, triangle a-b-c (1-2-3), a -- v=4, and the deleted edge (0,4).
# After the deletion u's only neighbour is a, so every hitting walk is
# u a (a loop around the triangle, either way, any number of times) v.
FIGURE8 = [(0, 4, 1.0), (0, 1, 1.0), (1, 2, 1.0), (2, 3, 1.0), (1, 3, 1.0), (1, 4, 1.0)]


def test_loop_erased_recovery_on_a_figure_eight(oracle_mod):
    """Whatever loops the winner ran, its loop erasure is u a v: the two edges
    (u,a), (a,v) are recovered in that order; without erasure every distinct
    edge of the winner's path is.  One walker, so the winner is whatever it
    did; seeds with looping winners must occur."""
    looped = 0
    for seed in range(60):
        res = {}
        for var in (0, oracle_mod.LOOP_ERASED):
            o = _oracle(oracle_mod, 5, FIGURE8, [(0, 4)], variant=var, s=1, L=12, seed=seed)
            r = o.apply_batch(Z, Z, ZW, np.array([0], np.uint32), np.array([4], np.uint32),
                              record_walkers=True)
            res[var] = (int(r["any_hit"][0]), int(r["walkers"]["steps"][0]),
                        o.last_recovered(0), _H(o))
            o.close()
        hit, steps, rec_le, H_le = res[oracle_mod.LOOP_ERASED]
        assert res[0][:2] == (hit, steps)  # the walks themselves are the same
        if not hit:
            continue
        assert rec_le == [(0, 1), (1, 4)]
        assert H_le == {(0, 1), (1, 4)}
        if steps > 2:
            looped += 1
            rec = res[0][2]
            # every hitting walk passes through a and then every triangle edge it used
            assert rec[0] == (0, 1) and rec[-1] == (1, 4) and len(rec) > 2
            assert set(rec) - {(0, 1), (1, 4)} <= {(1, 2), (2, 3), (3, 1), (2, 1), (3, 2), (1, 3)}
        else:
            assert res[0][2] == [(0, 1), (1, 4)]
    assert looped >= 3


def test_loop_erasure_keeps_loop_free_paths(oracle_mod):
    """G a 12-cycle, H the path 0..11: deleting (3,4) leaves G a path, where a
    non-backtracking walk cannot loop; the hitting walk 3 2 1 0 11 .. 4
    recovers the one G edge missing from H, (0,11), with or without
    erasure."""
    g = [(k, (k + 1) % 12, 1.0 + k) for k in range(12)]
    h = [(k, k + 1) for k in range(11)]
    got = []
    for var in (0, oracle_mod.LOOP_ERASED):
        o = _oracle(oracle_mod, 12, g, h, variant=var, s=4, L=12, seed=1)
        r = o.apply_batch(Z, Z, ZW, np.array([3], np.uint32), np.array([4], np.uint32))
        got.append((int(r["any_hit"][0]), o.last_recovered(0), _H(o)))
        o.close()
    assert got[0] == got[1]
    assert got[0][0] == 1 and got[0][1] == [(0, 11)]


def test_both_ends_on_a_star(oracle_mod):
    """Star with centre 0 and leaves 1..5, all in H; insertion (1,2), L = 2:
    a walker from one leaf goes to the centre, then to another leaf.  Even
    walkers start at 1 and hit iff they end at 2; odd walkers start at 2 and
    hit iff they end at 1."""
    star = [(0, k, float(k)) for k in range(1, 6)]
    o = _oracle(oracle_mod, 6, star, [(0, k) for k in range(1, 6)],
                variant=oracle_mod.BOTH_ENDS, s=64, L=2, seed=5)
    r = o.apply_batch(np.array([1], np.uint32), np.array([2], np.uint32), np.array([1.0]), Z, Z,
                      record_walkers=True)
    wk = r["walkers"]
    for k in range(64):
        start, target = (2, 1) if k % 2 else (1, 2)
        assert wk["steps"][k] == 2
        assert wk["end"][k] != start and wk["end"][k] != 0
        assert bool(wk["hit"][k]) == (wk["end"][k] == target), k
    assert wk["hit"][0::2].any() and wk["hit"][1::2].any()
    o.close()


def test_both_ends_deletion_walks_from_either_side(oracle_mod):
    """Figure eight, deletion (0,4): after it, 0 and 4 hang off a, so an even
    walker's first step is 0 -> 1 and an odd walker's is 4 -> 1; every hitting
    walker's path ends at the other endpoint, and its loop erasure is
    u a v or v a u."""
    o = _oracle(oracle_mod, 5, FIGURE8, [(0, 4)],
                variant=oracle_mod.BOTH_ENDS | oracle_mod.LOOP_ERASED, s=32, L=12, seed=9)
    r = o.apply_batch(Z, Z, ZW, np.array([0], np.uint32), np.array([4], np.uint32),
                      record_walkers=True)
    wk = r["walkers"]
    for k in range(32):
        if wk["hit"][k]:
            assert wk["end"][k] == (0 if k % 2 else 4)
    win = int(r["winner"][0])
    assert r["any_hit"][0]
    assert o.last_recovered(0) == ([(4, 1), (1, 0)] if win % 2 else [(0, 1), (1, 4)])
    o.close()


def test_two_stage_repairs_H_before_the_insertion_walks(oracle_mod):
    """G = 4-cycle 0-1-2-3-0, H = path 0-1-2-3.  Deleting (1,2) forces the walk
    1 0 3 2, which recovers (0,3).  The insertion (0,2) in the same batch:
    on the deferred snapshot (H = {01, 23}) its walkers die at the leaf 1
    and it is kept; with the repair first (H = {01, 23, 03}, 03 heavy) its
    walkers reach 2 through 3 and it is rejected."""
    g = [(0, 1, 1.0), (1, 2, 1.0), (2, 3, 1.0), (0, 3, 9.0)]
    h = [(0, 1), (1, 2), (2, 3)]
    out = {}
    for var in (0, oracle_mod.TWO_STAGE):
        o = _oracle(oracle_mod, 4, g, h, variant=var, s=8, L=6, seed=2)
        r = o.apply_batch(np.array([0], np.uint32), np.array([2], np.uint32), np.array([1.0]),
                          np.array([1], np.uint32), np.array([2], np.uint32))
        out[var] = (r["flag"].tolist(), r["any_hit"].tolist(), o.last_recovered(0), _H(o))
        o.close()
    # the deletion is the same either way
    assert out[0][2] == out[oracle_mod.TWO_STAGE][2] == [(0, 3)]
    assert out[0][0] == [1, 1] and out[0][1] == [0, 1]
    assert out[0][3] == {(0, 1), (2, 3), (0, 3), (0, 2)}
    assert out[oracle_mod.TWO_STAGE][0] == [0, 1] and out[oracle_mod.TWO_STAGE][1] == [1, 1]
    assert out[oracle_mod.TWO_STAGE][3] == {(0, 1), (2, 3), (0, 3)}


@pytest.mark.parametrize("var_name", ["TWO_STAGE", "LOOP_ERASED"])
def test_variant_without_its_case_changes_nothing(oracle_mod, var_name):
    """Insertion-only batches: no deletion repair, so neither the two-stage
    order nor loop erasure can change anything."""
    var = getattr(oracle_mod, var_name)
    wl = W.make_workload("grid64", side=24, ins=80, batches=3)
    rp, col, w = W.to_csr(wl.G.n, wl.G.u, wl.G.v, wl.G.w)
    res = []
    for v in (0, var):
        o = oracle_mod.Oracle(wl.G.n, rp, col, w, wl.hu, wl.hv, seed=wl.seed_walk, s=16, L=16,
                              variant=v)
        rs = [o.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv)["flag"].tolist() for b in wl.batches]
        res.append((rs, _H(o)))
        o.close()
    assert res[0] == res[1]


def test_unknown_variant_is_refused(oracle_mod):
    with pytest.raises(oracle_mod.OracleError):
        _oracle(oracle_mod, 5, FIGURE8, [(0, 4)], variant=8)
