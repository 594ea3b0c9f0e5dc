#!/usr/bin/env python3
"""Throughput of the dyGRASS update path on one MI355X.

A step is one batch through the whole path: validation, phase 1 (deletions
leave G and H), the walk kernel (insertion walks on H, deletion walks on G),
recovery/fallback, and phase 4 (G += insertions, H += accepted + recovered).
Inputs are uploaded to GPU memory before timing (device-resident batches via
dyg_apply_batch_dev); every step ends with a host synchronisation, as in the
plain one-launch-sequence-per-batch form.

Default workload: 1024x1024 circuit-like grid (1,048,576 vertices, 2,095,104
edges, lognormal(0,1) weights), maximum spanning forest + 10% off-tree edges
as the initial sparsifier, batches of 20,000 local insertions (2-6 hops),
64 walkers per update, step limit 32, no distortion threshold.

Prints one JSON line.  The walk kernel's roofline figure uses its algorithmic
gathered bytes (counted per step from the live degree of the vertex left) over
its duration measured with HIP events on its launch stream.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "updates/s + walker-steps/s (frac of HBM gather roofline); p50/p99 batch latency"
HBM_PEAK_GBS = 8000.0
KERNELS = {"plain": "k_walks", "batched": "k_walk_queue"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "walk_traffic.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("dyg_kernels.hip", "dyg_internal.h", "dyg_philox.h"):
        with open(os.path.join(ROOT, "paper_2505_02741_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, form: str):
    """HBM bytes per walk launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        d = json.load(f).get(f"{workload}/{form}")
    if not d or d.get("kernel_source") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_baseline(wl, batches, budget_s=20.0):
    """The CPU oracle as it stands, timed on this host's cores over the first
    batches of the same stream (as many as fit in about budget_s)."""
    import oracle
    from paper_2505_02741_amd import workloads as W

    rp, col, w = W.to_csr(wl.G.n, wl.G.u, wl.G.v, wl.G.w)
    o = oracle.Oracle(wl.G.n, rp, col, w, wl.hu, wl.hv, seed=wl.seed_walk, s=wl.s, L=wl.L,
                      K=wl.K)
    n_upd = 0
    t_all = 0.0
    done = 0
    for b in batches:
        t0 = time.perf_counter()
        o.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, s=b.s, L=b.L)
        t_all += time.perf_counter() - t0
        n_upd += b.size
        done += 1
        if t_all > budget_s:
            break
    steps = o.steps_total
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    o.close()
    return {
        "value": n_upd / t_all,
        "unit": "updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {done} batches ({n_upd} updates, {steps} walker steps) of the "
                  f"same stream from the initial state; C oracle, OpenMP over updates",
        "walker_steps_per_s": steps / t_all,
        "seconds": t_all,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="grid1024")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before the workload, copy this many MiB device to device once "
                         "(a known-size kernel for scaling rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    ap.add_argument("--form", choices=["both", "plain", "batched"], default="both",
                    help="plain: one wavefront per update; batched: persistent work-queue "
                         "walks; both: time both, report the batched one")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not "
              "supported (the multi-GPU sharding is a design, not a run).", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import numpy as np
    import torch

    from paper_2505_02741_amd import dygrass as D
    from paper_2505_02741_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.calibrate_copy_mib:
        nbytes = args.calibrate_copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy calibration: {nbytes} bytes read, {nbytes} bytes written",
              file=sys.stderr, flush=True)
        del src, dst
    n_batches = args.warmup + args.steps
    t0 = time.perf_counter()
    wl = W.make_workload(args.workload, seed=args.seed, n_batches=n_batches)
    t_gen = time.perf_counter() - t0
    print(f"# workload {args.workload}: n={wl.G.n} m={wl.G.m} H0={int(wl.h_mask.sum())} "
          f"batches={n_batches} gen={t_gen:.1f}s", file=sys.stderr, flush=True)
    rp, col, w = W.to_csr(wl.G.n, wl.G.u, wl.G.v, wl.G.w)

    def to_dev(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)

    dev_batches = []
    for b in wl.batches:
        db = dict(iu=to_dev(b.iu, np.int32), iv=to_dev(b.iv, np.int32),
                  iw=to_dev(b.iw, np.float64), du=to_dev(b.du, np.int32),
                  dv=to_dev(b.dv, np.int32),
                  s=None if b.s is None else to_dev(b.s.astype(np.int16), np.int16),
                  L=None if b.L is None else to_dev(b.L.astype(np.int16), np.int16),
                  L_max=int(b.L.max()) if b.L is not None and b.size else 0,
                  s_max=int(b.s.max()) if b.s is not None and b.size else 0,
                  results=torch.empty(b.size * 24, dtype=torch.uint8, device=dev))
        dev_batches.append(db)
    torch.cuda.synchronize()

    def run_form(flags):
        ctx = D.Dygrass(wl.G.n, rp, col, w, wl.hu, wl.hv, seed=wl.seed_walk, K=wl.K, s=wl.s,
                        L=wl.L, flags=D.FLAG_TIMING | flags)

        def step(i):
            db = dev_batches[i]
            D.dyg_apply_batch_dev(ctx.ctx, db["iu"], db["iv"], db["iw"], db["du"], db["dv"],
                                  s=db["s"], L=db["L"], L_max=db["L_max"], s_max=db["s_max"],
                                  results=db["results"])
            D.dyg_sync(ctx.ctx)

        for i in range(args.warmup):
            step(i)
        st0 = ctx.stats()
        torch.cuda.synchronize()
        lat = []
        t_start = time.perf_counter()
        for i in range(args.warmup, n_batches):
            ts = time.perf_counter()
            step(i)
            lat.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        t_total = time.perf_counter() - t_start
        st1 = ctx.stats()
        ctx.close()
        r = dict(t_total=t_total, lat=lat)
        for k in ("walk_steps", "walk_alg_bytes", "walk_ms_total", "walk_launches"):
            r[k] = st1[k] - st0[k]
        return r

    forms = {"plain": 0, "batched": D.FLAG_BATCHED}
    chosen = list(forms) if args.form == "both" else [args.form]
    runs = {}
    for name in chosen:
        runs[name] = run_form(forms[name])
        print(f"# {name}: {runs[name]['t_total'] / args.steps * 1e3:.3f} ms/step", file=sys.stderr,
              flush=True)
    head = "batched" if "batched" in runs else chosen[0]
    R = runs[head]
    updates = sum(b.size for b in wl.batches[args.warmup:])
    t_total, lat = R["t_total"], R["lat"]
    steps_walk = R["walk_steps"]
    alg_bytes = R["walk_alg_bytes"]
    walk_ms = R["walk_ms_total"]
    launches = R["walk_launches"]
    avg_walk_s = walk_ms / 1e3 / max(launches, 1)
    bytes_per_launch = alg_bytes / max(launches, 1)
    achieved = bytes_per_launch / avg_walk_s / 1e9 if avg_walk_s > 0 else 0.0
    traffic = measured_traffic(args.workload, head)
    cfg = wl.meta["cfg"]
    out = {
        "metric": METRIC,
        "value": updates / t_total,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_total / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {cfg['kind']} side {cfg.get('side')} "
                        f"(n={wl.G.n}, m={wl.G.m}), weights {cfg['weights']}, "
                        f"batches of {cfg.get('ins')} insertions + {cfg.get('dels')} deletions, "
                        f"s={wl.s}, L={wl.L}, K=inf, {head} form, one launch sequence and "
                        f"one host sync per batch",
            "global_batch": int(updates / args.steps),
            "parallelism": "single GPU",
        },
        "walker_steps_per_s": steps_walk / t_total,
        "walk_kernel_steps_per_s": steps_walk / (walk_ms / 1e3) if walk_ms > 0 else None,
        "p50_batch_ms": percentile(lat, 0.5) * 1e3,
        "p99_batch_ms": percentile(lat, 0.99) * 1e3,
        "walk_kernel_ms_avg": avg_walk_s * 1e3,
        "form": head,
        "forms": {k: {"updates_per_s": updates / v["t_total"],
                      "ms_per_step": v["t_total"] / args.steps * 1e3,
                      "walk_kernel_ms_avg": v["walk_ms_total"] / max(v["walk_launches"], 1),
                      "p50_batch_ms": percentile(v["lat"], 0.5) * 1e3,
                      "p99_batch_ms": percentile(v["lat"], 0.99) * 1e3}
                  for k, v in runs.items()},
        "roofline": {
            "bound": "hbm",
            "kernel": KERNELS[head],
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "alg_bytes_per_launch": bytes_per_launch,
            "alg_bytes_per_step": alg_bytes / max(steps_walk, 1),
        },
        "cpu_baseline": None,
    }
    if rank == 0 and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, wl.batches)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
