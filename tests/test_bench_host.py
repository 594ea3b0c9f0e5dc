"""Host-side logic of bench.py (no GPU): the counter-run parsing behind
`roofline.traffic`, the kernel-code key that ties counter runs to the source,
the labels of the walk kernels, and the refusal of more than one GPU."""
from __future__ import annotations

import csv
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def write_counters(path, counter, rows):
    """A rocprofv3 counter CSV with the columns bench.py reads."""
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, kib in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})


def test_code_key_ignores_comments_only(bench):
    a = "int f(int x) { return x + 1; }  // add one\n/* block */"
    b = "// a different comment\nint f(int x) {\n  return x + 1;\n}"
    c = "int f(int x) { return x + 2; }"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)


def test_traffic_from_counters_scales_by_the_copy(bench, tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    calib = 256 << 20
    # the copy kernel reads half its bytes as FETCH_SIZE and all of them as WRITE_SIZE
    fetch = [("__amd_rocclr_copyBuffer", calib / 2 / 1024), ("__amd_rocclr_copyBuffer", 1.0),
             ("void dyg::k_walks<false, false>(dyg::BatchArgs const* const*)", 1000.0),
             ("void dyg::k_walks<false, false>(dyg::BatchArgs const* const*)", 3000.0),
             ("dyg::k_walk_head<false>(dyg::BatchArgs const* const*)", 50.0)]
    write = [("__amd_rocclr_copyBuffer", calib / 1024),
             ("void dyg::k_walks<false, false>(dyg::BatchArgs const* const*)", 10.0),
             ("void dyg::k_walks<false, false>(dyg::BatchArgs const* const*)", 30.0)]
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    write_counters(fp, "FETCH_SIZE", fetch)
    write_counters(wp, "WRITE_SIZE", write)
    bench.traffic_from_counters(str(fp), str(wp), "k_walks", calib, "grid1024", "plain")
    d = json.load(open(tmp_path / "traffic.json"))["grid1024/plain"]
    assert d["fetch_scale"] == pytest.approx(2.0)
    assert d["write_scale"] == pytest.approx(1.0)
    assert d["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 1024 * 2.0)
    assert d["write_bytes_per_launch"] == pytest.approx(20.0 * 1024)
    assert d["launches"] == [2, 2]
    assert d["kernel_source"] == bench.kernel_source_hash()


def test_traffic_window_takes_the_last_dispatches(bench, tmp_path, monkeypatch):
    """The timed batches are the last ones: a window of 1 reads only the last
    dispatch of the kernel (warmup dispatches before it are ignored)."""
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    calib = 256 << 20
    k = "void dyg::k_walks<false, false>(dyg::BatchArgs const* const*)"
    fetch = [("__amd_rocclr_copyBuffer", calib / 1024), (k, 1000.0), (k, 3000.0)]
    write = [("__amd_rocclr_copyBuffer", calib / 1024), (k, 10.0), (k, 30.0)]
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    write_counters(fp, "FETCH_SIZE", fetch)
    write_counters(wp, "WRITE_SIZE", write)
    bench.traffic_from_counters(str(fp), str(wp), "k_walks", calib, "grid1024", "plain", window=1)
    d = json.load(open(tmp_path / "traffic.json"))["grid1024/plain"]
    assert d["fetch_bytes_per_launch"] == pytest.approx(3000.0 * 1024)
    assert d["write_bytes_per_launch"] == pytest.approx(30.0 * 1024)
    assert d["launches"] == [1, 1]


def test_traffic_of_a_two_kernel_walk_sums_per_launch(bench, tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    calib = 1 << 20
    head = "dyg::k_walk_head<false>(dyg::BatchArgs const* const*)"
    tail = "dyg::k_walk_tail<false>(dyg::BatchArgs const* const*, unsigned int)"
    fetch = [("__amd_rocclr_copyBuffer", calib / 1024), (head, 100.0), (head, 300.0), (tail, 10.0),
             (tail, 30.0)]
    write = [("__amd_rocclr_copyBuffer", calib / 1024), (head, 1.0), (head, 1.0), (tail, 2.0),
             (tail, 2.0)]
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    write_counters(fp, "FETCH_SIZE", fetch)
    write_counters(wp, "WRITE_SIZE", write)
    bench.traffic_from_counters(str(fp), str(wp), "k_walk_head+k_walk_tail", calib, "rmat22",
                                "batched")
    d = json.load(open(tmp_path / "traffic.json"))["rmat22/batched"]
    assert d["fetch_bytes_per_launch"] == pytest.approx((200.0 + 20.0) * 1024)
    assert d["write_bytes_per_launch"] == pytest.approx((1.0 + 2.0) * 1024)


def test_missing_kernel_is_an_error(bench, tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    write_counters(fp, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 512.0)])
    write_counters(wp, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 1024.0)])
    with pytest.raises(SystemExit):
        bench.traffic_from_counters(str(fp), str(wp), "k_walks", 1 << 20, "grid1024", "plain")


def test_walk_kernel_labels(bench):
    assert bench.walk_kernels("plain", None) == "k_walks"
    assert bench.walk_kernels("batched", {"tail_lanes": 8, "updates_per_wave": 4}) == \
        "k_walk_head+k_walk_tail"
    assert bench.walk_kernels("batched", {"tail_lanes": 0, "updates_per_wave": 4}) == "k_walk_range"
    assert bench.walk_kernels("batched", {"tail_lanes": 0, "updates_per_wave": 0}) == "k_walk_queue"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
