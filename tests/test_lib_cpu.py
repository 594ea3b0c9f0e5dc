"""CPU-side checks of the C ABI library: it is built, loads, and exports every
function include/dygrass.h declares (no compute calls: no GPU here)."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dygrass.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(dyg_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("dyg_init", "dyg_apply_batch", "dyg_query_sparsifier", "dyg_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2505_02741_amd import dygrass as D

    lib = ctypes.CDLL(D.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(D.EXPORTS) == set(declared_functions())


def test_binding_layouts_match_header():
    from paper_2505_02741_amd import dygrass as D

    assert ctypes.sizeof(D.dyg_params) == 56
    assert D.UPDATE_RESULT_DTYPE.itemsize == 24
    assert D.WALKER_RECORD_DTYPE.itemsize == 16
    p = D.dyg_default_params()
    assert p.Q == 24 and p.s_default == 64 and p.L_default == 32 and np.isinf(p.K)
    assert D.dyg_error_string(-5) == "inserted edge already in the graph"


def test_error_codes_agree_with_oracle():
    import oracle
    from paper_2505_02741_amd import dygrass as D

    for code, name in oracle.ERRORS.items():
        assert D.STATUS[code] == name


def test_product_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2505_02741_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "dyg_oracle" not in text, f


def test_missing_library_fails_loudly(tmp_path):
    """Without the built library the binding refuses to import: there is no
    fallback path."""
    import subprocess
    import sys

    env = dict(os.environ, DYGRASS_LIB=str(tmp_path / "absent" / "libdygrass.so"))
    r = subprocess.run([sys.executable, "-c", "import paper_2505_02741_amd.dygrass"], cwd=ROOT,
                       env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "is not built" in r.stderr


def test_flag_values_match_header():
    from paper_2505_02741_amd import dygrass as D

    text = open(os.path.join(ROOT, "include", "dygrass.h")).read()
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define DYG_FLAG_(\w+) (\d+)u", text)}
    assert defs == {"LEAN_POOLS": 1, "TIMING": 2, "BATCHED": 4, "GRAPH": 8, "AUTOTUNE": 16,
                    "TIMING_WALK": 32, "FAIL_POOL_GROWTH": 64, "BOTH_ENDS": 128,
                    "LOOP_ERASED": 256, "TWO_STAGE": 512}
    for name, v in defs.items():
        assert getattr(D, "FLAG_" + name) == v, name


def test_host_batch_lengths_are_checked_before_the_library_reads_them():
    import pytest

    from paper_2505_02741_amd import dygrass as D

    z = np.zeros(0)
    for args, kw in ((([0, 1], [2], [1.0, 1.0], z, z), {}),
                     (([0], [2], [1.0, 2.0], z, z), {}),
                     ((z, z, z, [0, 1], [2]), {}),
                     (([0], [2], [1.0], [3], [4]), {"s": [8]}),
                     (([0], [2], [1.0], [3], [4]), {"L": [8, 8, 8]})):
        with pytest.raises(ValueError):
            D.dyg_apply_batch(None, *args, **kw)  # refused before any library call


def test_device_batch_checks():
    import pytest
    import torch

    from paper_2505_02741_amd import dygrass as D

    def batch(n_ins=3, n_del=2, **over):
        b = dict(iu=torch.zeros(n_ins, dtype=torch.int32), iv=torch.ones(n_ins, dtype=torch.int32),
                 iw=torch.ones(n_ins, dtype=torch.float64),
                 du=torch.zeros(n_del, dtype=torch.int32), dv=torch.ones(n_del, dtype=torch.int32),
                 s=torch.full((n_ins + n_del,), 8, dtype=torch.int16),
                 L=torch.full((n_ins + n_del,), 8, dtype=torch.int16),
                 results=torch.zeros(24 * (n_ins + n_del), dtype=torch.uint8))
        b.update(over)
        return b

    # the forms the tests and the benchmark hand over are accepted
    D.check_dev_batch(**batch(), on_gpu=False)
    D.check_dev_batch(**batch(n_del=0, du=torch.zeros(0, dtype=torch.int32),
                              dv=torch.zeros(0, dtype=torch.int32), s=None, L=None,
                              results=None), on_gpu=False)
    D.check_dev_batch(**batch(s=0x7000, L=0x8000, results=0x9000), on_gpu=False)  # raw addresses
    bad = [dict(iu=torch.zeros(3, dtype=torch.int64)),          # 8-byte ids
           dict(iv=torch.ones(2, dtype=torch.int32)),           # short
           dict(iw=torch.ones(3, dtype=torch.float32)),         # 4-byte weights
           dict(iw=torch.ones(3, dtype=torch.int64)),           # integer weights
           dict(dv=torch.ones(3, dtype=torch.int32)),           # long
           dict(s=torch.full((5,), 8, dtype=torch.int32)),      # 4-byte walker counts
           dict(L=torch.full((4,), 8, dtype=torch.int16)),      # short
           dict(results=torch.zeros(24 * 5 - 1, dtype=torch.uint8)),
           dict(iu=torch.zeros(6, dtype=torch.int32)[::2])]     # not contiguous
    for over in bad:
        with pytest.raises(ValueError):
            D.check_dev_batch(**batch(**over), on_gpu=False)
    with pytest.raises(ValueError, match="GPU memory"):
        D.check_dev_batch(**batch())  # host tensors where device memory is required


def test_init_and_serving_inputs_are_checked_before_the_library_reads_them():
    import types

    import pytest

    from paper_2505_02741_amd import dygrass as D

    p = D.dyg_default_params()
    rp, col, w = [0, 1, 2], [1, 0], [1.0, 1.0]  # one edge on two vertices
    for args in (([0, 1], col, w, [0], [1]),          # rowptr short of n + 1
                 (rp, [1], w, [0], [1]),              # col short of rowptr[n]
                 (rp, col, [1.0], [0], [1]),          # w short of rowptr[n]
                 (rp, col, w, [0], [1, 0])):          # h_u, h_v differ
        with pytest.raises(ValueError):
            D.dyg_init(2, *args, p)
    srv = types.SimpleNamespace(h=None, _keep={})  # refused before the handle is used
    with pytest.raises(ValueError):
        D.DygServer.submit(srv, 0, [0, 1], [2], [1.0, 1.0], [], [])
