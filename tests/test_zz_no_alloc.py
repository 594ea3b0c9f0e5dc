"""dyg_apply_batch_dev_static (working memory in the library's static device
array, no allocation) against dyg_apply_batch_dev on the same batches: equal
per-update results and equal graphs after each batch, over two calls in a
row, the second with a smaller batch.  The size limit and the busy guard are
host-side refusals (nothing is launched)."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2505_02741_amd import workloads as W

from gpu_helpers import close_R, compare_state, make_pair, say

pytestmark = pytest.mark.gpu

BATCHED = 4  # DYG_FLAG_BATCHED


def _dev(torch, a, dt):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to("cuda:0")


def _batch_tensors(torch, b):
    kw = dict(iu=_dev(torch, b.iu, np.int32), iv=_dev(torch, b.iv, np.int32),
              iw=_dev(torch, b.iw, np.float64), du=_dev(torch, b.du, np.int32),
              dv=_dev(torch, b.dv, np.int32))
    if b.s is not None:
        kw.update(s=_dev(torch, b.s.astype(np.int16), np.int16), s_max=int(b.s.max()))
    if b.L is not None:
        kw.update(L=_dev(torch, b.L.astype(np.int16), np.int16), L_max=int(b.L.max()))
    return kw


def _two_batches():
    """A mesh stream whose second batch is smaller than its first, with uneven
    walker counts and step limits."""
    wl = W.make_workload("mesh128", side=12, ins=300, dels=200, batches=2)
    rng = np.random.default_rng(5)
    small = wl.batches[1]
    keep_i, keep_d = 40, 30
    small.iu, small.iv, small.iw = small.iu[:keep_i], small.iv[:keep_i], small.iw[:keep_i]
    small.du, small.dv = small.du[:keep_d], small.dv[:keep_d]
    for b in wl.batches:
        b.s = rng.integers(1, 97, b.size).astype(np.uint16)
        b.L = rng.integers(1, 33, b.size).astype(np.uint16)
    assert wl.batches[1].size < wl.batches[0].size
    return wl


@pytest.mark.parametrize("flags", [0, BATCHED])
def test_static_matches_dev(flags):
    import torch

    from paper_2505_02741_amd import dygrass as D

    wl = _two_batches()
    o, d_ref = make_pair(wl, flags=flags)
    o2, d_st = make_pair(wl, flags=flags)
    try:
        for t, b in enumerate(wl.batches):
            say(f"  static batch {t} flags={flags}: ins={b.n_ins} del={b.n_del}")
            kw = _batch_tensors(torch, b)
            res_ref = torch.zeros(b.size * 24, dtype=torch.uint8, device="cuda:0")
            res_st = torch.full((b.size * 24,), 0xAB, dtype=torch.uint8, device="cuda:0")
            D.dyg_apply_batch_dev(d_ref.ctx, results=res_ref, **kw)
            D.dyg_sync(d_ref.ctx)
            D.dyg_apply_batch_dev_static(d_st.ctx, results=res_st, **kw)
            D.dyg_sync(d_st.ctx)
            a = res_ref.cpu().numpy().view(D.UPDATE_RESULT_DTYPE)
            z = res_st.cpu().numpy().view(D.UPDATE_RESULT_DTYPE)
            for key in ("kind", "flag", "any_hit", "winner", "n_rec", "steps"):
                bad = np.flatnonzero(a[key] != z[key])
                assert bad.size == 0, f"batch {t} {key} differs at {bad[:10]}"
            assert close_R(a["Rmin"], z["Rmin"]), t
            # both contexts also agree with the oracle
            ro = o.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, s=b.s, L=b.L)
            o2.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, s=b.s, L=b.L)
            for key in ("flag", "any_hit", "winner", "n_rec", "steps"):
                assert np.array_equal(z[key], ro[key]), (t, key)
            compare_state(o, d_ref, f"dev {t}")
            compare_state(o2, d_st, f"static {t}")
        assert d_st.stats()["uid_base"] == d_ref.stats()["uid_base"]
    finally:
        d_ref.close()
        d_st.close()
        o.close()
        o2.close()


def test_static_refusals():
    """Refused on the host before anything is launched: a batch too large for
    the static array, a second static batch while one is in flight (same or
    another context on the GPU)."""
    import torch

    from paper_2505_02741_amd import dygrass as D

    wl = W.make_workload("grid64", batches=1)
    o, d1 = make_pair(wl)
    o2, d2 = make_pair(wl)
    try:
        # 100k deletions with step limits up to 1024 need gigabytes of slots
        n_big = 100_000
        z32 = torch.zeros(n_big, dtype=torch.int32, device="cuda:0")
        e32 = torch.zeros(0, dtype=torch.int32, device="cuda:0")
        e64 = torch.zeros(0, dtype=torch.float64, device="cuda:0")
        Lt = torch.full((n_big,), 1024, dtype=torch.int16, device="cuda:0")
        with pytest.raises(D.DygError) as ei:
            D.dyg_apply_batch_dev_static(d1.ctx, e32, e32, e64, z32, z32, L=Lt, L_max=1024)
        assert ei.value.name == "TOO_LARGE"
        b = wl.batches[0]
        kw = _batch_tensors(torch, b)
        res = torch.zeros(b.size * 24, dtype=torch.uint8, device="cuda:0")
        D.dyg_apply_batch_dev_static(d1.ctx, results=res, **kw)
        with pytest.raises(D.DygError) as ei:  # this context: not synced yet
            D.dyg_apply_batch_dev_static(d1.ctx, results=res, **kw)
        assert ei.value.name == "BUSY"
        with pytest.raises(D.DygError) as ei:  # another context, same GPU
            D.dyg_apply_batch_dev_static(d2.ctx, results=res, **kw)
        assert ei.value.name == "BUSY"
        D.dyg_sync(d1.ctx)
        ro = o.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, s=b.s, L=b.L)
        rl = res.cpu().numpy().view(D.UPDATE_RESULT_DTYPE)
        for key in ("flag", "any_hit", "steps"):
            assert np.array_equal(rl[key], ro[key]), key
        compare_state(o, d1, "after refusals")
        # the array is free again once the batch is synced
        D.dyg_apply_batch_dev_static(d2.ctx, results=res, **kw)
        D.dyg_sync(d2.ctx)
        o2.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, s=b.s, L=b.L)
        compare_state(o2, d2, "second context")
    finally:
        d1.close()
        d2.close()
        o.close()
        o2.close()
