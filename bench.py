#!/usr/bin/env python3
"""Throughput of the dyGRASS update path on one MI355X.

A step is one batch through the whole path: validation, phase 1 (deletions
leave G and H), the walk kernel (insertion walks on H, deletion walks on G),
recovery/fallback, and phase 4 (G += insertions, H += accepted + recovered).
The batches are in GPU memory before the timed region starts (device-resident
batches via dyg_apply_batch_dev); every step ends with a host
synchronisation.  The same batches are also run through dyg_apply_batch from
host arrays (upload and result download inside each step) and reported
beside the headline as the PCIe-inclusive rate.

Default workload (the headline line): R-MAT scale 22 (4,194,304 vertices,
edge factor 16, a=0.57 b=0.19 c=0.19, deduplicated, undirected), weights
U[1,10), maximum spanning forest + 10% off-tree edges as the initial
sparsifier, batches of log-uniform size 100..200,000 (70% local insertions,
30% deletions), walkers 16..128 and step limits 8..32 drawn per update, no
distortion threshold, in its own form: batched (the whole batch on the
device, each batch's launch sequence replayed from a captured hipGraph; the
walk schedule is --schedule, by default lockstep: one wavefront per update,
the fastest of the schedules on every batch of this stream, or the
autotuner's pick with --autotune).  The plain form (one wavefront per update,
launched directly) is timed on the same batches.
--workload grid1024 / mesh128 run the other configurations (plain form).

--form serving runs the many-graph serving workload instead (Poisson arrivals,
fused rounds, p50/p99 latency) against the plain form on the same requests.
--gwalk-stress runs one synthetic batch of 200,000 deletions of sparsifier
edges on the R-MAT graph: every deletion walks the 2 GB original graph.

Prints one JSON line.  The walk kernel's roofline figure uses its algorithmic
gathered bytes (counted per step from the live degree of the vertex left) over
its duration measured with HIP events on its launch stream (two per batch,
around the walk kernel only: DYG_FLAG_TIMING_WALK), over the timed batches.
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
# batched-form walk schedules (dyg_tuning: blocks per CU, refill, updates per
# wavefront, tail lanes, lockstep)
SCHEDULES = {"lockstep": (8, 1, 4, 0, 1), "range": (8, 8, 4, 0, 0),
             "headtail": (8, 1, 4, 8, 0), "queue": (8, 16, 0, 0, 0)}
# each configuration's own execution form
OWN_FORM = {"grid64": "plain", "grid1024": "plain", "mesh128": "plain", "rmat22": "batched"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "walk_traffic.json")


def walk_kernels(form: str, tuning) -> str:
    """The walk kernels a run of this form launched (the batched form's kept
    schedule decides which)."""
    if form != "batched" or not tuning:
        return KERNELS[form]
    if tuning.get("lockstep"):
        return KERNELS["plain"]
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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, batches, budget_s=15.0):
    """The CPU oracle as it stands, timed on this host: first with every
    thread OpenMP is given (OMP_NUM_THREADS, else all cores), over the first
    half of the stream at most, then with one thread over the next batches,
    each leg until about budget_s of CPU work (the stream runs on from the
    initial state)."""
    import oracle
    from paper_2505_02741_amd import workloads as W

    rp, col, w = W.to_csr(wl.G.n, wl.G.u, wl.G.v, wl.G.w)
    t0 = time.perf_counter()
    o = oracle.Oracle(wl.G.n, rp, col, w, wl.hu, wl.hv, seed=wl.seed_walk, s=wl.s, L=wl.L,
                      K=wl.K)
    t_init = time.perf_counter() - t0
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads_all = int(os.environ.get("OMP_NUM_THREADS", nproc or 1))
    legs = []
    it = iter(enumerate(batches))
    half = max(len(batches) // 2, 1)  # the all-thread leg leaves the rest to one thread
    for threads in (threads_all, 1):
        oracle.set_threads(threads)
        n_upd = steps0 = 0
        t_all = 0.0
        first = last = None
        steps0 = o.steps_total
        for i, b in it:
            t1 = time.perf_counter()
            o.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, s=b.s, L=b.L)
            t_all += time.perf_counter() - t1
            n_upd += b.size
            first = i if first is None else first
            last = i
            if t_all > budget_s or (threads != 1 and i + 1 >= half):
                break
        if first is None:
            break
        legs.append(dict(threads=threads, updates=n_upd, seconds=t_all,
                         steps=o.steps_total - steps0, batches=(first, last)))
    o.close()
    main = legs[0]
    out = {
        "value": main["updates"] / main["seconds"],
        "unit": "updates/s",
        "cores": main["threads"],
        "kind": "oracle",
        "sample": f"batches {main['batches'][0]}-{main['batches'][1]} ({main['updates']} "
                  f"updates, {main['steps']} walker steps) of the same stream from the initial "
                  f"state; C oracle, OpenMP over the updates of a batch, "
                  f"{main['threads']} threads",
        "walker_steps_per_s": main["steps"] / main["seconds"],
        "seconds": main["seconds"],
        "nproc": nproc,
        "cpu_model": cpu_model(),
        "oracle_init_s": t_init,
    }
    if len(legs) > 1:
        one = legs[1]
        out["one_thread"] = {
            "value": one["updates"] / one["seconds"], "unit": "updates/s", "cores": 1,
            "sample": f"batches {one['batches'][0]}-{one['batches'][1]} ({one['updates']} "
                      f"updates, {one['steps']} walker steps), continuing the same stream",
            "walker_steps_per_s": one["steps"] / one["seconds"], "seconds": one["seconds"]}
    return out


def traffic_from_counters(fetch_csv, write_csv, kernel, calib_bytes, workload, form, window=0):
    """Per-launch HBM bytes of `kernel` from two rocprofv3 --pmc runs of the
    same bench command (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each
    scaled so that the copy kernel of calib_bytes (the --calibrate-copy-mib
    run) reads and writes exactly calib_bytes (that copy is told from the
    workload's small copies by size: its counters read at least a quarter of
    calib_bytes); averaged over the last `window` dispatches of the kernel
    (the bench's timed batches; 0 = all), written to the traffic file."""

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
    if window:
        # rows come in dispatch order: the timed batches are the last ones
        f_vals = {k: v[-window:] for k, v in f_vals.items()}
        w_vals = {k: v[-window:] for k, v in w_vals.items()}
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


def run_stream(D, torch, wl, rp, col, w, dev_batches, flags, warmup, tuning=None, host=False):
    """Apply every batch in order on a fresh context (buffers reserved for the
    largest batch); time all but the first `warmup` batches.  host: each step
    hands host arrays to dyg_apply_batch, which uploads the batch and
    downloads its per-update results inside the step."""
    t0 = time.perf_counter()
    ctx = D.Dygrass(wl.G.n, rp, col, w, wl.hu, wl.hv, seed=wl.seed_walk, K=wl.K, s=wl.s,
                    L=wl.L, flags=D.FLAG_TIMING_WALK | flags)
    reserve_for(D, ctx, wl.batches)
    t_init = time.perf_counter() - t0
    if tuning:
        D.dyg_set_tuning(ctx.ctx, *tuning)

    def step(i):
        if host:
            b = wl.batches[i]
            ctx.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, s=b.s, L=b.L)
            return
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
    r = dict(t_total=t_total, lat=lat, tuning=tuning_kept, h_edges_end=st1["h_edges"],
             t_init=t_init)
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
    own = OWN_FORM[args.workload]
    head = args.form if args.form in ("plain", "batched") else own
    graph = args.graph if args.graph is not None else (head == "batched")
    autotune = bool(args.autotune) and head == "batched"
    if args.warmup is None:
        args.warmup = TUNE_CANDIDATES if args.workload == "rmat22" else 2
    if autotune and args.warmup < TUNE_CANDIDATES:
        args.warmup = TUNE_CANDIDATES
    n_batches = args.warmup + args.steps
    t0 = time.perf_counter()
    wl = W.make_workload(args.workload, seed=args.seed, n_batches=n_batches)
    print(f"# workload {args.workload}: n={wl.G.n} m={wl.G.m} H0={int(wl.h_mask.sum())} "
          f"batches={n_batches} gen={time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    rp, col, w = W.to_csr(wl.G.n, wl.G.u, wl.G.v, wl.G.w)
    dev_batches = [to_device(np, torch, dev, b) for b in wl.batches]
    torch.cuda.synchronize()

    batched_flags = D.FLAG_BATCHED | (D.FLAG_AUTOTUNE if autotune else 0)
    flags = {"plain": 0, "batched": batched_flags | (D.FLAG_GRAPH if graph else 0)}
    chosen = [head] if args.form in ("plain", "batched") else ["plain", "batched"]
    # the batched form's walk schedule: the autotuner's pick, else --schedule
    tuning = {"plain": None, "batched": None if autotune else SCHEDULES[args.schedule]}
    runs = {}
    for name in chosen:
        runs[name] = run_stream(D, torch, wl, rp, col, w, dev_batches, flags[name], args.warmup,
                                tuning=tuning[name])
        print(f"# {name}: {runs[name]['t_total'] / args.steps * 1e3:.3f} ms/step "
              f"(context init {runs[name]['t_init']:.1f}s)", file=sys.stderr, flush=True)
    if "batched" in runs:  # the other legs of the batched form keep its schedule
        k = runs["batched"]["tuning"]
        tuning["batched"] = (k["walk_blocks_per_cu"], k["refill_min"], k["updates_per_wave"],
                             k["tail_lanes"], k["lockstep"])
        flags["batched"] &= ~D.FLAG_AUTOTUNE
    # the walk kernel inside a captured graph is not timed: the roofline of the
    # batched form then comes from the same schedule launched directly
    if head == "batched" and graph:
        timed = run_stream(D, torch, wl, rp, col, w, dev_batches, D.FLAG_BATCHED, args.warmup,
                           tuning=tuning["batched"])
        print(f"# batched, direct launches (walk timing): "
              f"{timed['t_total'] / args.steps * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
    else:
        timed = runs[head]
    pcie = None
    if not args.no_pcie:
        pcie = run_stream(D, torch, wl, rp, col, w, dev_batches, flags[head], args.warmup,
                          tuning=tuning[head], host=True)
        print(f"# {head}, host arrays (PCIe inside each step): "
              f"{pcie['t_total'] / args.steps * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
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
    kernel = walk_kernels(head, timed.get("tuning"))
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
    if head == "batched":
        sched = ("schedule autotuned on the warmup batches" if autotune else
                 f"{args.schedule} walk schedule")
        form_text = ("batched form (whole batch on the device, " + sched +
                     (", launch sequence replayed from a captured hipGraph" if graph else "") +
                     "), one host sync per batch")
    else:
        form_text = "plain form, one launch sequence and one host sync per batch"
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
                        f"{cfg['weights']}, {stream}, {walk}, K=inf, {form_text}; batches "
                        f"resident in GPU memory",
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
            "kernel": kernel,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(args.workload, head),
            "alg_bytes_per_launch": bytes_per_launch,
            "alg_bytes_per_step": alg_bytes / max(steps_walk, 1),
            "launches": launches,
        },
        "cpu_baseline": None,
    }
    if pcie is not None:
        out["pcie_inclusive"] = {"updates_per_s": updates / pcie["t_total"],
                                 "ms_per_step": pcie["t_total"] / args.steps * 1e3,
                                 "p50_batch_ms": percentile(pcie["lat"], 0.5) * 1e3,
                                 "p99_batch_ms": percentile(pcie["lat"], 0.99) * 1e3}
    # off-tree density of the sparsifier (Sec. IV metric): edges beyond the
    # initial spanning forest F per vertex, (|E_H| - |F|) / |V| (|F| = n - 1
    # on a connected graph), before the stream and after its last batch (read
    # after the timed region)
    forest = wl.meta["forest_edges"]
    out["d_H"] = {"initial": (int(wl.h_mask.sum()) - forest) / wl.G.n,
                  "end": (R["h_edges_end"] - forest) / wl.G.n}
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


def main_gwalk_stress(args):
    """One batch of 200,000 deletions drawn uniformly from the sparsifier's
    edges of the R-MAT scale-22 graph, walkers 16..128 and step limits 8..32
    per update: every deletion walks the original graph (about 2 GB of rows,
    well beyond the 256 MB cache), so the walk kernel reads HBM.  A warmup
    batch of 2,000 other such deletions comes first.  Reports the walk kernel
    alone (HIP events) against its algorithmic gathered bytes."""
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
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t0 = time.perf_counter()
    wl = W.make_workload("rmat22", seed=args.seed, n_batches=0)
    rng = np.random.default_rng(np.random.SeedSequence([args.seed, 0x6A1C]))
    n_del, n_warm = 200_000, 2_000
    h_idx = np.flatnonzero(wl.h_mask)
    pick = rng.choice(h_idx, n_del + n_warm, replace=False)
    batches = []
    for sel in (pick[:n_warm], pick[n_warm:]):
        b = W.Batch(np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.float64),
                    wl.G.u[sel].astype(np.uint32), wl.G.v[sel].astype(np.uint32))
        b.s = rng.integers(16, 129, b.size).astype(np.uint16)
        b.L = rng.integers(8, 33, b.size).astype(np.uint16)
        batches.append(b)
    wl.batches = batches
    print(f"# gwalk stress: n={wl.G.n} m={wl.G.m} gen={time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    rp, col, w = W.to_csr(wl.G.n, wl.G.u, wl.G.v, wl.G.w)
    dev_batches = [to_device(np, torch, dev, b) for b in batches]
    form = args.form if args.form in ("plain", "batched") else "plain"
    flags = D.FLAG_BATCHED if form == "batched" else 0
    r = run_stream(D, torch, wl, rp, col, w, dev_batches, flags, 1)
    walk_s = r["walk_ms_total"] / 1e3 / max(r["walk_launches"], 1)
    achieved = r["walk_alg_bytes"] / max(r["walk_launches"], 1) / walk_s / 1e9 if walk_s else 0
    out = {
        "metric": METRIC,
        "value": n_del / r["t_total"],
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": r["t_total"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"gwalk_stress: R-MAT scale 22 (n={wl.G.n}, m={wl.G.m}), one "
                               f"batch of {n_del} deletions of sparsifier edges (walks on the "
                               f"original graph), s=16-128, L=8-32 per update, {form} form",
                   "global_batch": n_del, "parallelism": "single GPU"},
        "walk_kernel_ms": walk_s * 1e3,
        "walk_steps": r["walk_steps"],
        "walk_kernel_steps_per_s": r["walk_steps"] / walk_s if walk_s else None,
        "roofline": {"bound": "hbm", "kernel": walk_kernels(form, r.get("tuning")),
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("gwalk_stress", form),
                     "alg_bytes_per_launch": r["walk_alg_bytes"] / max(r["walk_launches"], 1),
                     "alg_bytes_per_step": r["walk_alg_bytes"] / max(r["walk_steps"], 1)},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed batches first (default: 10 on rmat22, the autotuner's "
                         "trial count, so that the timed batches are the same with or "
                         "without it; 2 elsewhere)")
    ap.add_argument("--workload", default="rmat22",
                    choices=["grid64", "grid1024", "mesh128", "rmat22"])
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pcie", action="store_true",
                    help="skip the host-array (PCIe-inclusive) run of the same batches")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before the workload, copy this many MiB device to device once "
                         "(a known-size kernel for scaling rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    ap.add_argument("--form", choices=["both", "plain", "batched", "serving"], default="both",
                    help="plain: one wavefront per update; batched: walker-packed walk; both: "
                         "time both, report the workload's own form; serving: the many-graph "
                         "serving workload")
    ap.add_argument("--graph", action=argparse.BooleanOptionalAction, default=None,
                    help="batched form: replay each batch's launch sequence from a captured "
                         "hipGraph (one per power-of-two size class); default on for a "
                         "workload whose own form is batched")
    ap.add_argument("--schedule", choices=sorted(SCHEDULES), default="lockstep",
                    help="batched form's walk schedule when not autotuned: lockstep (one "
                         "wavefront per update, as the plain form walks; the fastest on "
                         "every workload measured), range, headtail or queue")
    ap.add_argument("--autotune", action=argparse.BooleanOptionalAction, default=False,
                    help="batched form: the first batches try the autotuner's schedules "
                         f"(warmup raised to at least {TUNE_CANDIDATES} so that they are "
                         "not timed) and the best is kept, instead of --schedule")
    ap.add_argument("--gwalk-stress", action="store_true",
                    help="one synthetic batch of 200,000 deletions of sparsifier edges on "
                         "the R-MAT graph (every deletion walks the original graph)")
    ap.add_argument("--graphs", type=int, default=64, help="serving: resident graphs")
    ap.add_argument("--requests-per-graph", type=int, default=16)
    ap.add_argument("--max-nodes", type=int, default=500_000)
    ap.add_argument("--max-fused", type=int, default=32)
    ap.add_argument("--max-inflight", type=int, default=2)
    ap.add_argument("--mem-budget", type=int, default=16, help="serving: GiB for batches in flight")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic file from two rocprofv3 counter runs of this "
                         "command (with --calibrate-copy-mib) instead of running")
    ap.add_argument("--traffic-kernel", default=None,
                    help="with --traffic-from: the walk kernel(s) to read ('a+b' sums two); "
                         "default: the form's default schedule")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only; --gpus {args.gpus} is not "
              "supported (sharding over several GPUs is designed, not implemented).",
              file=sys.stderr)
        sys.exit(2)
    if args.traffic_from:
        # the form the measured run used (the stress run defaults to plain)
        form = (args.form if args.form in KERNELS else
                "plain" if args.gwalk_stress else OWN_FORM[args.workload])
        kernel = args.traffic_kernel or KERNELS[form]
        traffic_from_counters(args.traffic_from[0], args.traffic_from[1], kernel,
                              args.calibrate_copy_mib << 20,
                              "gwalk_stress" if args.gwalk_stress else args.workload, form,
                              window=1 if args.gwalk_stress else args.steps)
        return
    if args.form == "serving":
        main_serving(args)
    elif args.gwalk_stress:
        main_gwalk_stress(args)
    else:
        main_batches(args)


if __name__ == "__main__":
    main()
