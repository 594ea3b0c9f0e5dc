"""Full-size parity: the workloads at their real sizes, in the launch
configurations the benchmark times (plain and batched forms, device-resident
batches), against the CPU oracle on every batch.  Per-update results and the final edge
sets are compared exactly; per-walker records on the first batch."""
from __future__ import annotations

import time

import numpy as np
import pytest

from paper_2505_02741_amd import workloads as W

from gpu_helpers import close_R, compare_state, make_pair, say

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

BATCHED = 4
FORMS = pytest.mark.parametrize("flags", [0, BATCHED], ids=["plain", "batched"])


def _device_batch(D, torch, d, b, dev):
    def T(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)

    res = torch.zeros(b.size * 24, dtype=torch.uint8, device=dev)
    kw = {}
    if b.s is not None:
        kw = dict(s=T(b.s.astype(np.int16), np.int16), L=T(b.L.astype(np.int16), np.int16),
                  L_max=int(b.L.max()), s_max=int(b.s.max()))
    D.dyg_apply_batch_dev(d.ctx, T(b.iu, np.int32), T(b.iv, np.int32), T(b.iw, np.float64),
                          T(b.du, np.int32), T(b.dv, np.int32), results=res, **kw)
    D.dyg_sync(d.ctx)
    return res.cpu().numpy().view(D.UPDATE_RESULT_DTYPE)


def _run_full(name, flags, n_batches=None, walker_batches=(0,), **over):
    import torch

    from paper_2505_02741_amd import dygrass as D

    dev = torch.device("cuda:0")
    t0 = time.time()
    wl = W.make_workload(name, n_batches=n_batches, **over)
    say(f"{name}: n={wl.G.n} m={wl.G.m} H0={int(wl.h_mask.sum())} gen {time.time() - t0:.1f}s")
    o, d = make_pair(wl, flags=flags)
    try:
        for t, b in enumerate(wl.batches):
            t1 = time.time()
            if t in walker_batches:
                ro = o.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, s=b.s, L=b.L,
                                   record_walkers=True)
                rl, wk = d.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, s=b.s, L=b.L, walkers=True)
                for key in ("hit", "steps", "end"):
                    assert np.array_equal(wk[key], ro["walkers"][key]), (t, key)
                assert close_R(wk["R"], ro["walkers"]["R"])
            else:
                ro = o.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, s=b.s, L=b.L)
                rl = _device_batch(D, torch, d, b, dev)
            for key in ("flag", "any_hit", "winner", "n_rec", "steps"):
                bad = np.flatnonzero(rl[key] != ro[key])
                assert bad.size == 0, f"batch {t} {key} differs at {bad[:8]}"
            assert close_R(rl["Rmin"], ro["Rmin"]), t
            say(f"  batch {t}: ins {b.n_ins} del {b.n_del} kept {int(ro['flag'][:b.n_ins].sum())} "
                f"steps {int(ro['steps'].sum())} ({time.time() - t1:.1f}s)")
        compare_state(o, d, name)
        st = d.stats()
        assert st["walk_steps"] == o.steps_total
        assert st["walk_alg_bytes"] == o.alg_bytes_total
        assert st["uid_base"] == o.uid_base
    finally:
        d.close()
        o.close()


@FORMS
def test_grid1024_all_batches(flags):
    """1024x1024 lognormal grid, 10 x 20,000 insertions, s=64, L=32."""
    _run_full("grid1024", flags)


@FORMS
def test_mesh128_all_batches(flags):
    """128^3 FEM mesh, 20 x (10,000 insertions + 10,000 deletions), s=64, L=24."""
    _run_full("mesh128", flags)


@FORMS
def test_rmat_scale18_uneven_batches(flags):
    """R-MAT scale 18 (edge factor 16), 12 uneven batches (100..20,000
    updates, 70/30), per-update s in 16..128 and L in 8..32."""
    _run_full("rmat22", flags, scale=18, batches=12, size_hi=20_000)


@pytest.mark.timeout(1200)
def test_rmat22_full_scale_first_batches():
    """R-MAT scale 22 at its real size (4,194,304 vertices, 64M edges, rows up
    to ~163k entries, above 65,535), the first four batches of its stream
    (238, 191, 382 and 172,011 updates: a batch of more than 150,000, with
    hash tables and fallback slots at that size), in the plain form, the
    batched form and the benchmark's configuration (batched, lockstep walk,
    captured graphs) side by side, against one oracle, per-update results of
    every batch and both edge sets at the end."""
    import torch

    from paper_2505_02741_amd import dygrass as D

    dev = torch.device("cuda:0")
    t0 = time.time()
    wl = W.make_workload("rmat22", n_batches=4)
    deg = np.bincount(np.r_[wl.G.u, wl.G.v], minlength=wl.G.n)
    say(f"rmat22: n={wl.G.n} m={wl.G.m} max degree {int(deg.max())} H0={int(wl.h_mask.sum())} "
        f"batches {[b.size for b in wl.batches]} gen {time.time() - t0:.1f}s")
    assert deg.max() > 65535
    assert max(b.size for b in wl.batches) >= 150_000
    import oracle

    rp, col, w = W.to_csr(wl.G.n, wl.G.u, wl.G.v, wl.G.w)
    say(f"  CSR built ({time.time() - t0:.1f}s)")
    o = oracle.Oracle(wl.G.n, rp, col, w, wl.hu, wl.hv, seed=wl.seed_walk, K=wl.K, s=wl.s,
                      L=wl.L)
    say(f"  oracle ready ({time.time() - t0:.1f}s)")
    d_plain = D.Dygrass(wl.G.n, rp, col, w, wl.hu, wl.hv, seed=wl.seed_walk, K=wl.K, s=wl.s,
                        L=wl.L, flags=0)
    say(f"  plain context ready ({time.time() - t0:.1f}s)")
    d_batched = D.Dygrass(wl.G.n, rp, col, w, wl.hu, wl.hv, seed=wl.seed_walk, K=wl.K, s=wl.s,
                          L=wl.L, flags=BATCHED)
    say(f"  batched context ready ({time.time() - t0:.1f}s)")
    # the benchmark's launch configuration: batched form, lockstep walk,
    # every batch replayed from a captured graph
    d_bench = D.Dygrass(wl.G.n, rp, col, w, wl.hu, wl.hv, seed=wl.seed_walk, K=wl.K, s=wl.s,
                        L=wl.L, flags=BATCHED | D.FLAG_GRAPH)
    D.dyg_set_tuning(d_bench.ctx, 8, 1, 4, 0, lockstep=1)
    say(f"  batched lockstep graph context ready ({time.time() - t0:.1f}s)")
    ctxs = (("plain", d_plain), ("batched", d_batched), ("batched lockstep graph", d_bench))
    try:
        for t, b in enumerate(wl.batches):
            t1 = time.time()
            ro = o.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, s=b.s, L=b.L)
            for tag, d in ctxs:
                rl = _device_batch(D, torch, d, b, dev)
                for key in ("flag", "any_hit", "winner", "n_rec", "steps"):
                    bad = np.flatnonzero(rl[key] != ro[key])
                    assert bad.size == 0, f"{tag} batch {t} {key} differs at {bad[:8]}"
                assert close_R(rl["Rmin"], ro["Rmin"]), (tag, t)
            say(f"  batch {t}: ins {b.n_ins} del {b.n_del} kept "
                f"{int(ro['flag'][:b.n_ins].sum())} recovered {int(ro['n_rec'].sum())} "
                f"steps {int(ro['steps'].sum())} ({time.time() - t1:.1f}s)")
        for tag, d in ctxs:
            compare_state(o, d, f"rmat22 {tag}")
            st = d.stats()
            assert st["walk_steps"] == o.steps_total
            assert st["walk_alg_bytes"] == o.alg_bytes_total
            say(f"  {tag}: state equal to the oracle's ({time.time() - t0:.1f}s)")
    finally:
        d_plain.close()
        d_batched.close()
        d_bench.close()
        o.close()
