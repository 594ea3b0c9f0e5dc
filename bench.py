#!/usr/bin/env python3
"""Throughput of the dyGRASS update path on one MI355X.

A step is one batch through the whole path: validation, phase 1 (deletions
leave G and H), the walk kernel (insertion walks on H, deletion walks on G),
recovery/fallback, and phase 4 (G += insertions, H += accepted + recovered).
Batches are uploaded to GPU memory before timing (device-resident batches via
dyg_apply_batch_dev); every step ends with a host synchronisation.

Default workload (the headline line): 1024x1024 circuit-like grid (1,048,576
vertices, 2,095,104 edges, lognormal(0,1) weights), maximum spanning forest +
10% off-tree edges as the initial sparsifier, batches of 20,000 local
insertions (2-6 hops), 64 walkers per update, step limit 32, no distortion
threshold, in the plain form (one launch sequence and one host sync per
batch).  The batched form (each wavefront walks the walkers of a few
consecutive updates, lanes refilled as walkers stop) is timed on the same
batches for comparison.

--form serving runs the many-graph serving workload instead (Poisson arrivals,
fused rounds, p50/p99 latency) against the plain form on the same requests.

Prints one JSON line.  The walk kernel's roofline figure uses its algorithmic
gathered bytes (counted per step from the live degree of the vertex left) over
its duration measured with HIP events on its launch stream (two per batch,
around the walk kernel only: DYG_FLAG_TIMING_WALK).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "updates/s + walker-steps/s (frac of HBM gather roofline); p50/p99 batch latency"
HBM_PEAK_GBS = 8000.0
# the walk kernels of each form ("a+b": a walk of two launches, summed)
KERNELS = {"plain": "k_walks", "batched": "k_walk_head+k_walk_tail"}
TUNE_CANDIDATES = 10  # schedules the autotuner tries, one batch each
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "walk_traffic.json")


def walk_kernels(form: str, tuning) -> str:
    """The walk kernels a run of this form launched (the batched form's kept
    schedule decides which)."""
    if form != "batched" or not tuning:
        return KERNELS[form]
    if tuning["tail_lanes"] > 0:
        return "k_walk_head+k_walk_tail"
    return "k_walk_range" if tuning["updates_per_wave"] > 0 else "k_walk_queue"


def _code_only(text: str) -> str:
    """C++ source without comments and with whitespace collapsed (the kernel
    sources hold no string literals), so that comment edits keep the hash."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(read=None) -> str:
    """Hash of the walk kernels' code (comments ignored): counter runs are
    reported only while it is unchanged."""
    h = hashlib.sha256()
    for f in ("dyg_kernels.hip", "dyg_internal.h", "dyg_philox.h"):
        if read is None:
            with open(os.path.join(ROOT, "paper_2505_02741_amd", "csrc", f)) as fh:
                text = fh.read()
        else:
            text = read(f)
        h.update(_code_only(text).encode())
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


def traffic_from_counters(fetch_csv, write_csv, kernel, calib_bytes, workload, form):
    """Per-launch HBM bytes of `kernel` from two rocprofv3 --pmc runs of the
    same bench command (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each
    scaled so that the copy kernel of calib_bytes (the --calibrate-copy-mib
    run) reads and writes exactly calib_bytes (that copy is told from the
    workload's small copies by size: its counters read at least a quarter of
    calib_bytes); written to the traffic file."""

    names = kernel.split("+")

    def per_kernel(path, counter):
        vals, copy = {k: [] for k in names}, []
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"]) * 1024.0
                hit = [k for k in names if k + "<" in r["Kernel_Name"] or k + "(" in r["Kernel_Name"]]
                if hit:
                    vals[hit[0]].append(v)
                elif "copyBuffer" in r["Kernel_Name"] and v > 0.25 * calib_bytes:
                    copy.append(v)
        return vals, copy

    f_vals, f_copy = per_kernel(fetch_csv, "FETCH_SIZE")
    w_vals, w_copy = per_kernel(write_csv, "WRITE_SIZE")
    if not all(f_vals.values()) or not all(w_vals.values()) or not f_copy or not w_copy:
        raise SystemExit("traffic: kernel or calibration copy missing from the counter files")
    f_scale = calib_bytes / max(f_copy)
    w_scale = calib_bytes / max(w_copy)
    # one walk = one dispatch of each of its kernels
    fetch = sum(sum(v) / len(v) for v in f_vals.values()) * f_scale
    write = sum(sum(v) / len(v) for v in w_vals.values()) * w_scale
    d = {}
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    d[f"{workload}/{form}"] = {
        "kernel": kernel, "kernel_source": kernel_source_hash(),
        "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
        "bytes_per_launch": fetch + write, "fetch_scale": f_scale, "write_scale": w_scale,
        "launches": [min(len(v) for v in f_vals.values()), min(len(v) for v in w_vals.values())],
    }
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    print(json.dumps(d[f"{workload}/{form}"]))


def to_device(np, torch, dev, b):
    def T(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)

    return dict(iu=T(b.iu, np.int32), iv=T(b.iv, np.int32), iw=T(b.iw, np.float64),
                du=T(b.du, np.int32), dv=T(b.dv, np.int32),
                s=None if b.s is None else T(b.s.astype(np.int16), np.int16),
                L=None if b.L is None else T(b.L.astype(np.int16), np.int16),
                L_max=int(b.L.max()) if b.L is not None and b.size else 0,
                s_max=int(b.s.max()) if b.s is not None and b.size else 0,
                results=torch.empty(b.size * 24, dtype=torch.uint8, device=dev))


def reserve_for(D, ctx, batches):
    """Size the context's batch buffers for the largest batch of the stream."""
    D.dyg_reserve(ctx.ctx, max(b.n_ins for b in batches), max(b.n_del for b in batches),
                  max((int(b.s.max()) for b in batches if b.s is not None and b.size), default=0),
                  max((int(b.L.max()) for b in batches if b.L is not None and b.size), default=0))


def run_stream(D, torch, wl, rp, col, w, dev_batches, flags, warmup, tuning=None):
    """Apply every batch in order on a fresh context (buffers reserved for the
    largest batch); time all but the first `warmup` batches."""
    ctx = D.Dygrass(wl.G.n, rp, col, w, wl.hu, wl.hv, seed=wl.seed_walk, K=wl.K, s=wl.s,
                    L=wl.L, flags=D.FLAG_TIMING_WALK | flags)
    reserve_for(D, ctx, wl.batches)
    if tuning:
        D.dyg_set_tuning(ctx.ctx, *tuning)

    def step(i):
        db = dev_batches[i]
        D.dyg_apply_batch_dev(ctx.ctx, db["iu"], db["iv"], db["iw"], db["du"], db["dv"],
                              s=db["s"], L=db["L"], L_max=db["L_max"], s_max=db["s_max"],
                              results=db["results"])
        D.dyg_sync(ctx.ctx)

    for i in range(warmup):
        step(i)
    st0 = ctx.stats()
    torch.cuda.synchronize()
    lat = []
    t_start = time.perf_counter()
    for i in range(warmup, len(dev_batches)):
        ts = time.perf_counter()
        step(i)
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    st1 = ctx.stats()
    tuning_kept = D.dyg_get_tuning(ctx.ctx)
    ctx.close()
    r = dict(t_total=t_total, lat=lat, tuning=tuning_kept, h_edges_end=st1["h_edges"])
    for k in ("walk_steps", "walk_alg_bytes", "walk_ms_total", "walk_launches"):
        r[k] = st1[k] - st0[k]
    return r


def form_summary(runs, updates, steps):
    return {k: {"updates_per_s": updates / v["t_total"],
                "ms_per_step": v["t_total"] / steps * 1e3,
                "walk_kernel_ms_avg": (v["walk_ms_total"] / v["walk_launches"]
                                       if v["walk_launches"] else None),
                "p50_batch_ms": percentile(v["lat"], 0.5) * 1e3,
                "p99_batch_ms": percentile(v["lat"], 0.99) * 1e3}
            for k, v in runs.items()}


def main_batches(args):
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
    print(f"# workload {args.workload}: n={wl.G.n} m={wl.G.m} H0={int(wl.h_mask.sum())} "
          f"batches={n_batches} gen={time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    rp, col, w = W.to_csr(wl.G.n, wl.G.u, wl.G.v, wl.G.w)
    dev_batches = [to_device(np, torch, dev, b) for b in wl.batches]
    torch.cuda.synchronize()

    forms = {"plain": 0, "batched": D.FLAG_BATCHED | (D.FLAG_GRAPH if args.graph else 0) |
             (D.FLAG_AUTOTUNE if args.autotune else 0)}
    head = args.form if args.form in forms else ("plain" if args.workload != "rmat22" else "batched")
    chosen = [head] if args.form in forms else list(forms)
    runs = {}
    for name in chosen:
        runs[name] = run_stream(D, torch, wl, rp, col, w, dev_batches, forms[name], args.warmup)
        print(f"# {name}: {runs[name]['t_total'] / args.steps * 1e3:.3f} ms/step",
              file=sys.stderr, flush=True)
    # the walk kernel inside a captured graph is not timed: the roofline of the
    # batched form then comes from the same schedule launched directly
    if "batched" in runs and head == "batched" and args.graph:
        timed = run_stream(D, torch, wl, rp, col, w, dev_batches,
                           D.FLAG_BATCHED | (D.FLAG_AUTOTUNE if args.autotune else 0),
                           args.warmup)
    else:
        timed = runs[head]
    R = runs[head]
    updates = sum(b.size for b in wl.batches[args.warmup:])
    t_total, lat = R["t_total"], R["lat"]
    steps_walk = timed["walk_steps"]
    alg_bytes = timed["walk_alg_bytes"]
    walk_ms = timed["walk_ms_total"]
    launches = timed["walk_launches"]
    avg_walk_s = walk_ms / 1e3 / max(launches, 1)
    bytes_per_launch = alg_bytes / max(launches, 1)
    achieved = bytes_per_launch / avg_walk_s / 1e9 if avg_walk_s > 0 else 0.0
    cfg = wl.meta["cfg"]
    if cfg["kind"] == "rmat":
        shape = f"R-MAT scale {cfg['scale']} edge factor {cfg['ef']}"
    else:
        shape = f"{cfg['kind']} side {cfg.get('side')}"
    if cfg.get("size_lo"):
        stream = (f"batches of {cfg['size_lo']}-{cfg['size_hi']} updates (log-uniform, "
                  f"{int(cfg['ins_frac'] * 100)}% insertions)")
    else:
        stream = f"batches of {cfg.get('ins')} insertions + {cfg.get('dels')} deletions"
    walk = (f"s={cfg['s_lo']}-{cfg['s_hi']}, L={cfg['L_lo']}-{cfg['L_hi']} per update"
            if cfg.get("s_lo") else f"s={wl.s}, L={wl.L}")
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
            "workload": f"{args.workload}: {shape} (n={wl.G.n}, m={wl.G.m}), weights "
                        f"{cfg['weights']}, {stream}, {walk}, K=inf, {head} form, "
                        f"one launch sequence and one host sync per batch",
            "global_batch": int(updates / args.steps),
            "parallelism": "single GPU",
        },
        "walker_steps_per_s": steps_walk / t_total,
        "walk_kernel_steps_per_s": steps_walk / (walk_ms / 1e3) if walk_ms > 0 else None,
        "p50_batch_ms": percentile(lat, 0.5) * 1e3,
        "p99_batch_ms": percentile(lat, 0.99) * 1e3,
        "walk_kernel_ms_avg": avg_walk_s * 1e3,
        "form": head,
        "forms": form_summary(runs, updates, args.steps),
        "roofline": {
            "bound": "hbm",
            "kernel": walk_kernels(head, timed.get("tuning")),
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(args.workload, head),
            "alg_bytes_per_launch": bytes_per_launch,
            "alg_bytes_per_step": alg_bytes / max(steps_walk, 1),
        },
        "cpu_baseline": None,
    }
    # off-tree density of the sparsifier, |E_H| / |V| - 1 (Sec. IV metric),
    # before the stream and after its last batch (read after the timed region)
    out["d_H"] = {"initial": int(wl.h_mask.sum()) / wl.G.n - 1.0,
                  "end": R["h_edges_end"] / wl.G.n - 1.0}
    if "batched" in runs:
        out["batched_schedule"] = runs["batched"]["tuning"]
    if "plain" in runs and "batched" in runs:
        out["batched_over_plain"] = runs["plain"]["t_total"] / runs["batched"]["t_total"]
    if int(os.environ.get("RANK", "0")) == 0 and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, wl.batches)
    print(json.dumps(out), flush=True)


def main_serving(args):
    """Many resident graphs: the same requests through the plain form (one
    batch at a time per request) and through the serving engine (fused
    rounds), first all offered at once (saturation), then as Poisson
    arrivals at 0.7 x the saturated request rate (latency)."""
    import numpy as np
    import torch

    from paper_2505_02741_amd import dygrass as D
    from paper_2505_02741_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.zeros(1, device="cuda:0")
    t0 = time.perf_counter()
    fleet = W.make_fleet(n_graphs=args.graphs, seed=args.seed, n_hi=args.max_nodes,
                         batches_per_graph=args.requests_per_graph)
    n_req = sum(len(wl.batches) for wl in fleet)
    n_upd = sum(b.size for wl in fleet for b in wl.batches)
    print(f"# fleet: {len(fleet)} graphs, {sum(wl.G.m for wl in fleet)} edges, {n_req} requests, "
          f"{n_upd} updates, gen {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    csr = [W.to_csr(wl.G.n, wl.G.u, wl.G.v, wl.G.w) for wl in fleet]
    rng = np.random.default_rng(args.seed)
    # one global request order that keeps each graph's own order
    owner = np.repeat(np.arange(len(fleet)), [len(wl.batches) for wl in fleet])
    rng.shuffle(owner)
    order, nxt = [], [0] * len(fleet)
    for g in owner:
        order.append((int(g), nxt[g]))
        nxt[g] += 1

    def contexts(flags):
        out = [D.Dygrass(wl.G.n, *csr[g], wl.hu, wl.hv, seed=wl.seed_walk, K=wl.K, s=wl.s,
                         L=wl.L, flags=flags) for g, wl in enumerate(fleet)]
        for c, wl in zip(out, fleet):
            reserve_for(D, c, wl.batches)
        return out

    # plain: each request on its own graph, one launch sequence + host sync
    ctxs = contexts(0)
    plain_res, plain_lat = {}, []
    torch.cuda.synchronize()
    t_plain = time.perf_counter()
    for g, t in order:
        b = fleet[g].batches[t]
        ts = time.perf_counter()
        plain_res[(g, t)] = ctxs[g].apply_batch(b.iu, b.iv, b.iw, b.du, b.dv)[0]
        plain_lat.append(time.perf_counter() - ts)
    t_plain = time.perf_counter() - t_plain
    for c in ctxs:
        c.close()
    print(f"# plain: {n_upd / t_plain:.0f} updates/s", file=sys.stderr, flush=True)

    def serve(rate):
        ctxs = contexts(D.FLAG_BATCHED)
        srv = D.DygServer(mem_budget=args.mem_budget << 30, max_fused=args.max_fused,
                          max_inflight=args.max_inflight)
        gids = [srv.add_graph(c) for c in ctxs]
        owner_of, done = {}, []
        gaps = rng.exponential(1.0 / rate, len(order)) if rate else np.zeros(len(order))
        t_start = time.perf_counter()
        t_next = t_start
        for (g, t), gap in zip(order, gaps):
            t_next += gap
            while rate and time.perf_counter() < t_next:
                done += srv.poll()
            b = fleet[g].batches[t]
            owner_of[srv.submit(gids[g], b.iu, b.iv, b.iw, b.du, b.dv)] = (g, t)
            if not rate:
                continue
            done += srv.poll()
        done += srv.drain()
        elapsed = time.perf_counter() - t_start
        srv.close()
        for c in ctxs:
            c.close()
        bad = 0
        for r in done:
            key = owner_of[r["request_id"]]
            ref = plain_res[key]
            if r["status"] != 0:
                bad += 1
                continue
            for f in ("flag", "any_hit", "winner", "n_rec", "steps", "Rmin"):
                if not np.array_equal(r["results"][f], ref[f]):
                    bad += 1
                    break
        lat = [r["t_done"] - r["t_submit"] for r in done]
        return dict(elapsed=elapsed, lat=lat, mismatches=bad, n=len(done))

    sat = serve(0.0)
    sat_rate = n_req / sat["elapsed"]
    print(f"# serving, all offered: {n_upd / sat['elapsed']:.0f} updates/s", file=sys.stderr,
          flush=True)
    load = serve(0.7 * sat_rate)
    print(f"# serving, Poisson at 0.7x: {n_upd / load['elapsed']:.0f} updates/s", file=sys.stderr,
          flush=True)
    out = {
        "metric": METRIC,
        "value": n_upd / sat["elapsed"],
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": n_req,
        "warmup": 0,
        "ms_per_step": sat["elapsed"] / n_req * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"serving: {len(fleet)} graphs (grid / 3D mesh / R-MAT cycled, "
                        f"n log-uniform 10k-{args.max_nodes}), {n_req} requests of "
                        f"1-50,000 updates (log-uniform, 60% insertions), s=64, L=24, K=inf; "
                        f"fused rounds of up to {args.max_fused} requests, "
                        f"{args.max_inflight} rounds in flight",
            "global_batch": int(n_upd / n_req),
            "parallelism": "single GPU",
        },
        "form": "serving",
        "serving_all_offered": {"updates_per_s": n_upd / sat["elapsed"],
                                "p50_ms": percentile(sat["lat"], 0.5) * 1e3,
                                "p99_ms": percentile(sat["lat"], 0.99) * 1e3},
        "serving_poisson_0.7": {"offered_requests_per_s": 0.7 * sat_rate,
                                "updates_per_s": n_upd / load["elapsed"],
                                "p50_ms": percentile(load["lat"], 0.5) * 1e3,
                                "p99_ms": percentile(load["lat"], 0.99) * 1e3},
        "plain": {"updates_per_s": n_upd / t_plain,
                  "p50_ms": percentile(plain_lat, 0.5) * 1e3,
                  "p99_ms": percentile(plain_lat, 0.99) * 1e3},
        "serving_over_plain": t_plain / sat["elapsed"],
        "results_equal_plain": sat["mismatches"] == 0 and load["mismatches"] == 0,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="grid1024",
                    choices=["grid64", "grid1024", "mesh128", "rmat22"])
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before the workload, copy this many MiB device to device once "
                         "(a known-size kernel for scaling rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    ap.add_argument("--form", choices=["both", "plain", "batched", "serving"], default="both",
                    help="plain: one wavefront per update; batched: range walk; both: time "
                         "both, report the workload's own form; serving: the many-graph "
                         "serving workload")
    ap.add_argument("--graph", action="store_true",
                    help="batched form: replay each batch's launch sequence from a captured "
                         "hipGraph (one per power-of-two size class)")
    ap.add_argument("--autotune", action="store_true",
                    help="batched form: the first batches try the autotuner's schedules "
                         f"(warmup raised to at least {TUNE_CANDIDATES} so that they are "
                         "not timed)")
    ap.add_argument("--graphs", type=int, default=64, help="serving: resident graphs")
    ap.add_argument("--requests-per-graph", type=int, default=16)
    ap.add_argument("--max-nodes", type=int, default=500_000)
    ap.add_argument("--max-fused", type=int, default=32)
    ap.add_argument("--max-inflight", type=int, default=2)
    ap.add_argument("--mem-budget", type=int, default=16, help="serving: GiB for batches in flight")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic file from two rocprofv3 counter runs of this "
                         "command (with --calibrate-copy-mib) instead of running")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only; --gpus {args.gpus} is not "
              "supported (sharding over several GPUs is designed, not implemented).",
              file=sys.stderr)
        sys.exit(2)
    if args.autotune and args.warmup < TUNE_CANDIDATES:
        args.warmup = TUNE_CANDIDATES
    if args.traffic_from:
        form = args.form if args.form in KERNELS else "plain"
        traffic_from_counters(args.traffic_from[0], args.traffic_from[1], KERNELS[form],
                              args.calibrate_copy_mib << 20, args.workload, form)
        return
    if args.form == "serving":
        main_serving(args)
    else:
        main_batches(args)


if __name__ == "__main__":
    main()
