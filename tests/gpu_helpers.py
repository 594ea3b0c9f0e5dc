"""Shared helpers of the GPU parity tests: run the HIP library and the CPU
oracle side by side on the same seeded inputs and compare."""
from __future__ import annotations

import math
import sys

import numpy as np

from paper_2505_02741_amd import workloads as W

# Resistance sums: the contract is 1e-12 relative; the two sides add the same
# IEEE doubles in the same order, so they agree exactly in practice.
R_RTOL = 1e-12


# pytest's capture manager (set by the conftest fixture): progress lines of
# long GPU tests go straight to the real stdout, so a slow test shows that it
# is alive while pytest captures everything else
CAPMAN = None


def say(*a):
    if CAPMAN is not None:
        with CAPMAN.global_and_fixture_disabled():
            print(*a, flush=True)
    else:
        print(*a, flush=True)
    sys.stdout.flush()


# oracle variant bit -> library flag
VARIANT_FLAGS = {1: 128, 2: 256, 4: 512}


def make_pair(wl, *, K=None, dead_end=0, slack=0.5, Q=24, s=None, L=None, w_ref=0.0,
              uid_base=0, G=None, H=None, flags=0, variant=0):
    import oracle
    from paper_2505_02741_amd import dygrass as D

    if G is None:
        G = (wl.G.u, wl.G.v, wl.G.w)
    if H is None:
        H = (wl.hu, wl.hv)
    rp, col, w = W.to_csr(wl.G.n, *G)
    K = wl.K if K is None else K
    s = wl.s if s is None else s
    L = wl.L if L is None else L
    o = oracle.Oracle(wl.G.n, rp, col, w, H[0], H[1], seed=wl.seed_walk, K=K, s=s, L=L, Q=Q,
                      w_ref=w_ref, dead_end=dead_end, uid_base=uid_base, variant=variant)
    for bit, flag in VARIANT_FLAGS.items():
        if variant & bit:
            flags |= flag
    d = D.Dygrass(wl.G.n, rp, col, w, H[0], H[1], seed=wl.seed_walk, K=K, s=s, L=L, Q=Q,
                  w_ref=w_ref, dead_end=dead_end, slack=slack, uid_base=uid_base, flags=flags)
    return o, d


def close_R(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    # equal infinities (no hit) match; finite values within the relative
    # tolerance; anything else (finite against infinite, NaN) does not
    same_inf = np.isinf(a) & np.isinf(b) & (np.sign(a) == np.sign(b))
    if not np.all(same_inf | (np.isfinite(a) & np.isfinite(b))):
        return False
    fin = ~same_inf
    diff = np.abs(a[fin] - b[fin])
    tol = R_RTOL * np.maximum(np.abs(a[fin]), np.abs(b[fin]))
    return bool(np.all(diff <= tol))


def compare_batch(o, d, b, record=True, tag=""):
    ro = o.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, s=b.s, L=b.L, record_walkers=record)
    rl, wk = d.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, s=b.s, L=b.L, walkers=record)
    n_ins = b.n_ins
    kind = np.r_[np.zeros(n_ins, np.uint8), np.ones(b.n_del, np.uint8)]
    assert np.array_equal(rl["kind"], kind), tag
    for key in ("flag", "any_hit", "winner", "n_rec", "steps"):
        bad = np.flatnonzero(rl[key] != ro[key])
        assert bad.size == 0, f"{tag} {key} differs at updates {bad[:10]}: lib {rl[key][bad[:5]]} oracle {ro[key][bad[:5]]}"
    assert close_R(rl["Rmin"], ro["Rmin"]), tag
    if record:
        ow = ro["walkers"]
        for key in ("hit", "steps", "end"):
            bad = np.flatnonzero(wk[key] != ow[key])
            assert bad.size == 0, f"{tag} walker {key} differs at {bad[:10]}"
        assert close_R(wk["R"], ow["R"]), tag
    return ro, rl


def compare_state(o, d, tag=""):
    problem = d.check_state()
    assert problem == "", f"{tag}: device state inconsistent: {problem}"
    for which in ("G", "H"):
        ou, ov, ow = o.query(which)
        lu, lv, lw = d.query(which)
        assert ou.size == lu.size, f"{tag} {which} edge count {lu.size} vs oracle {ou.size}"
        assert np.array_equal(ou, lu) and np.array_equal(ov, lv), f"{tag} {which} edge sets differ"
        assert np.array_equal(ow, lw), f"{tag} {which} weights differ"


def run_parity(wl, batches=None, record=True, tag="", **kw):
    o, d = make_pair(wl, **kw)
    try:
        compare_state(o, d, tag + " init")
        for t, b in enumerate(wl.batches if batches is None else batches):
            say(f"  {tag} batch {t}: ins={b.n_ins} del={b.n_del}")
            compare_batch(o, d, b, record=record, tag=f"{tag} batch {t}")
            compare_state(o, d, f"{tag} batch {t}")
        st = d.stats()
        assert st["uid_base"] == o.uid_base
        assert st["walk_steps"] == o.steps_total
        assert st["walk_alg_bytes"] == o.alg_bytes_total
    finally:
        d.close()
        o.close()
