#!/usr/bin/env python
"""Throughput of the fast block AMG on one MI355X: solves/s and unknowns/s at
N = 2^20 intervals for the FP32 V-cycle + FP64 refinement form and the plain
FP64 form, with p50/p99 latency, the roofline of the finest-level FFT matvec
sweep, and the CPU FP64 oracle timed on the host beside it.

A step is one complete solve (outer residual, V-cycles over every level --
FFT matvecs, Jacobi, transfers, coarsest LU -- until ||r||/||r_0|| < tol) of
the synthetic manufactured problem u = x^2 (1-x)^2, constant kernel
3/(2 delta^3), delta = 0.25, zero volume constraint, with b resident in HBM.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
LAT_SAMPLES = 100      # solves behind each p50 / p99


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed solves per form")
    ap.add_argument("--warmup", type=int, default=3, help="untimed solves per form")
    ap.add_argument("--logN", type=int, default=20)
    ap.add_argument("--delta", type=float, default=0.25)
    ap.add_argument("--kernel", default="const", choices=["const", "weighted", "fractional"])
    ap.add_argument("--alpha", type=float, default=0.4)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pcg", action="store_true",
                    help="skip the V-cycle-preconditioned CG forms (reported beside the headline)")
    ap.add_argument("--prof-steps", type=int, default=3,
                    help="solves of the profiled pass (HIP events around the finest-level "
                         "passes, eager launches) that gives the roofline; 0 = skip")
    ap.add_argument("--batch", type=int, default=512,
                    help="instances of the uneven batch (seeded N, delta, kernel, random b) "
                         "solved together by amg_solve_batch beside the headline; 0 = skip")
    ap.add_argument("--no-c2", action="store_true",
                    help="skip the size/horizon/kernel sweep (N = 2^14, 2^17, 2^20; delta = 0.05, "
                         "0.25; constant and weighted kernels) beside the headline")
    ap.add_argument("--no-ext", action="store_true",
                    help="skip the extension forms (standard collocation with volume data, BDF4 "
                         "steps, the weakly singular model, GMRES, W-cycles) beside the headline")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the precision configuration (N = 2^22, fractional alpha = 0.4, "
                         "delta = 0.1, FP32 V-cycle + FP64 residual, CG) beside the headline")
    ap.add_argument("--no-deep-fold", action="store_true",
                    help="headline forms without AMG_FLAG_DEEP_FOLD (the cycle below the four-step "
                         "levels in the one-workgroup kernel rather than as one dense product)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default level geometries (no amg_autotune before the runs)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the serving run (Poisson arrivals, mixed sizes); 0 = skip")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="serving arrivals per second")
    ap.add_argument("--serve-budget-gb", type=float, default=96.0,
                    help="device memory budget of the request server")
    ap.add_argument("--serve-workers", type=int, default=2,
                    help="set-up threads of the server (each has its own stream; with the "
                         "server's and the arrival side's streams, 2 keep to the 4 hardware queues "
                         "a process gets by default)")
    ap.add_argument("--serve-small-log2", type=int, default=17,
                    help="requests with N <= 2^this run in a second lane of the server "
                         "(0: one lane)")
    ap.add_argument("--serve-small-rounds", type=int, default=4,
                    help="rounds of the small lane per round of the other requests")
    ap.add_argument("--serve-rounds", type=int, default=1,
                    help="rounds per amg_server_step of the serving run")
    ap.add_argument("--serve-queue-gb", type=float, default=48.0,
                    help="bound on the b and x vectors of requests submitted and not finished; "
                         "arrivals beyond it are shed (counted)")
    ap.add_argument("--serve-drain-s", type=float, default=60.0,
                    help="longest wait for requests still in flight after the last arrival")
    ap.add_argument("--pmc-driver", action="store_true",
                    help="the short program the --pmc counter runs profile: a plain copy of "
                         "known size, then two mixed solves of the workload (eager launches)")
    ap.add_argument("--pmc-batch-driver", action="store_true",
                    help="the program the batch --pmc runs profile: the uneven batch set up, a "
                         "plain copy of known size, then two batch solves")
    ap.add_argument("--batch-traffic-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="from the counter CSVs of two rocprofv3 --pmc runs of --pmc-batch-driver, "
                         "write one batch solve's HBM bytes to profiles/; no GPU needed")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="from the counter-collection CSVs of two rocprofv3 --pmc runs of "
                         "--pmc-driver (FETCH_SIZE, then WRITE_SIZE), write the finest FP32 "
                         "sweep's HBM traffic, scaled by the copy's, to profiles/; no GPU needed")
    ap.add_argument("--rocprof-summary", metavar="KERNEL_TRACE_CSV",
                    help="summarise a rocprofv3 --kernel-trace CSV (per kernel and grid size) "
                         "and exit; no GPU needed")
    return ap.parse_args()


def rocprof_summary(path):
    """Per (kernel, grid size) call count and average duration from a
    rocprofv3 kernel-trace CSV; grid size identifies the level."""
    import collections
    import csv
    rows = list(csv.DictReader(open(path)))
    agg = collections.defaultdict(lambda: [0, 0.0])
    for r in rows:
        name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("amg::", "")
        key = (name, int(r["Grid_Size_X"]))
        agg[key][0] += 1
        agg[key][1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    tot = sum(v[1] for v in agg.values())
    print(f"{'kernel':34s} {'grid':>9s} {'calls':>6s} {'avg_us':>9s} {'share%':>7s}")
    for (name, grid), (calls, us) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        if us / tot < 0.002:
            continue
        print(f"{name:34s} {grid:9d} {calls:6d} {us / calls:9.2f} {100 * us / tot:7.2f}")
    st = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows)
    print(f"total kernel time {tot / 1e3:.2f} ms over {len(rows)} dispatches")


COPY_BYTES = 256 << 20  # the PMC run's plain copy: reads and writes this many bytes
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fp32_finest_sweep_N2e20.json")
KERNEL_SOURCES = ["fourstep.hpp", "fourstep_f32.hip", "fft_lds.hpp", "kernel_common.hpp",
                  "amg_device.hpp"]


def kernel_source_hash():
    """Hash of the sources the finest-level FFT pass kernels are built from:
    a traffic measurement is valid only for the kernels it was taken on."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2202_11288_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def pmc_driver(args):
    import torch

    from paper_2202_11288_amd import binding as B
    x = torch.ones(COPY_BYTES // 4, device="cuda", dtype=torch.float32)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    del x, y
    N = 2 ** args.logN
    k = kernel_of(B, args)
    b = torch.from_numpy(B.amg_manufactured_rhs(k, args.delta, N)).cuda()
    h = B.amg_setup(k, args.delta, N,
                    B.amg_default_opts(precision=B.AMG_MIXED, flags=B.AMG_FLAG_EAGER))
    try:
        for _ in range(2):
            xs = torch.zeros_like(b)
            B.amg_solve(h, b, xs, args.tol)
        torch.cuda.synchronize()
    finally:
        B.amg_destroy(h)
    print("pmc driver done", flush=True)


BATCH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_batch_c4.json")


def pmc_batch_driver(args):
    """The program the batch --pmc runs profile: the uneven batch's handles
    are set up, then a plain copy of known size (its counter reading scales
    the others, and it marks where the solves start), then the batch is
    solved twice from x_0 = 0 (the bench's untimed and timed calls)."""
    import torch

    from paper_2202_11288_amd import binding as B
    inst = batch_instances(args.batch)
    opts = B.amg_default_opts(precision=B.AMG_MIXED, inner=B.AMG_INNER_PCG,
                              max_iter=BATCH_MAX_ITER)
    hs, bs, xs = [], [], []
    try:
        for d in inst:
            hs.append(B.amg_setup(batch_kernel(B, d), d["delta"], d["N"], opts))
            bs.append(torch.from_numpy(d["b"]).cuda())
            xs.append(torch.zeros_like(bs[-1]))
        torch.cuda.synchronize()
        x = torch.ones(COPY_BYTES // 4, device="cuda", dtype=torch.float32)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
        for _ in range(2):
            for v in xs:
                v.zero_()
            B.amg_solve_batch(hs, bs, xs, [args.tol] * len(hs),
                              allow=(B.AMG_OK, B.AMG_NOT_CONVERGED))
            torch.cuda.synchronize()
    finally:
        for h in hs:
            B.amg_destroy(h)
    print("pmc batch driver done", flush=True)


def batch_traffic_summary(fetch_csv, write_csv, args):
    """HBM bytes of one batch solve: FETCH_SIZE / WRITE_SIZE of every
    dispatch after the marker copy (the two solves), scaled by the copy's
    factor, halved."""
    import csv

    def load(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        key = "Dispatch_Id" if rows and "Dispatch_Id" in rows[0] else None
        if key:
            rows.sort(key=lambda r: int(r[key]))
        return rows

    out = {}
    for label, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = load(path, counter)
        vals = [float(r["Counter_Value"]) * 1024.0 for r in rows]
        copies = [i for i, r in enumerate(rows) if "copyBuffer" in r["Kernel_Name"]]
        mark = max(copies, key=lambda i: vals[i])
        scale = COPY_BYTES / vals[mark]
        after = vals[mark + 1:]
        out[label] = {"scale": round(scale, 4), "dispatches": len(after),
                      "bytes_per_batch": round(sum(after) * scale / 2)}
    res = {"kernel": "every dispatch of one amg_solve_batch call of the uneven batch",
           "workload": batch_workload_id(args),
           "source_hash": kernel_source_hash(),
           "fetch": out["fetch"], "write": out["write"],
           "bytes_per_batch": out["fetch"]["bytes_per_batch"] + out["write"]["bytes_per_batch"],
           "commands": [
               "cd /tmp && timeout -s KILL 240 rocprofv3 --pmc FETCH_SIZE --output-format csv "
               "-d <out>/pmc_bfetch -o run -- python3 <repo>/bench.py --pmc-batch-driver",
               "cd /tmp && timeout -s KILL 240 rocprofv3 --pmc WRITE_SIZE --output-format csv "
               "-d <out>/pmc_bwrite -o run -- python3 <repo>/bench.py --pmc-batch-driver",
               "python bench.py --batch-traffic-summary <out>/pmc_bfetch/run_counter_collection.csv "
               "<out>/pmc_bwrite/run_counter_collection.csv"]}
    with open(BATCH_TRAFFIC_FILE, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


def measured_batch_traffic(args):
    try:
        with open(BATCH_TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash() or t.get("workload") != batch_workload_id(args):
        return None
    return t.get("bytes_per_batch")


def traffic_workload(args):
    """The workload a traffic measurement belongs to (the --pmc-driver run)."""
    return {"logN": args.logN, "kernel": args.kernel, "delta": args.delta,
            "alpha": args.alpha if args.kernel == "fractional" else None}


def traffic_summary(fetch_csv, write_csv, logN, workload):
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the finest-level FP32
    FFT pass kernels, each scaled by the factor that maps the same counter's
    reading for the plain copy onto the copy's known bytes; per sweep = the
    sum over the three passes' dispatches divided by the number of sweeps."""
    import collections
    import csv
    import re

    def load(path, counter):
        per = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            name = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "")
            per[(name, int(r["Grid_Size"]))].append(float(r["Counter_Value"]) * 1024.0)
        return per

    out = {}
    for label, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        per = load(path, counter)
        copies = [v for (name, g), vals in per.items() if "copyBuffer" in name for v in vals]
        big = max(copies)
        scale = COPY_BYTES / big
        # the finest level's FP32 passes: the wide (512-thread) column tiles and
        # the row pass on rows of 2048 points (KR = 8); other levels may share
        # the template arguments or the grid size, not both: the largest grid
        # among the matching instances is the finest level's
        finest = {"k_col_fwd": ("amg::k_col_fwd<float", ", 16, 512,"),
                  "k_row": ("amg::k_row<float", ", 8, 0>"),
                  "k_col_inv": ("amg::k_col_inv<float", ", 16, 512,")}
        sel = {}
        for kind, (pre, tag) in finest.items():
            keys = [(name, g) for (name, g) in per if name.startswith(pre) and tag in name]
            gmax = max((g for _, g in keys), default=0)
            sel[kind] = [x for (name, g) in keys if g == gmax for x in per[(name, g)]]
        sweeps = len(sel["k_row"])
        if not sweeps or any(len(v) != sweeps for v in sel.values()):
            raise SystemExit(f"{counter}: finest-level dispatch counts differ: "
                             f"{ {k: len(v) for k, v in sel.items()} }")
        total = sum(sum(v) for v in sel.values()) * scale / sweeps
        out[label] = {"copy_counter_bytes": big, "copy_known_bytes": COPY_BYTES,
                      "scale": round(scale, 4), "sweeps": sweeps,
                      "bytes_per_sweep": round(total),
                      "per_pass_bytes": {k: round(sum(v) * scale / sweeps) for k, v in sel.items()}}
    res = {"kernel": f"fp32 finest-level FFT matvec sweep (3 passes), N=2^{logN}",
           "workload": workload,
           "source_hash": kernel_source_hash(),
           "fetch": out["fetch"], "write": out["write"],
           "traffic_bytes_per_sweep": out["fetch"]["bytes_per_sweep"] + out["write"]["bytes_per_sweep"],
           "commands": [
               "cd /tmp && timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE --output-format csv "
               "-d <out>/pmc_fetch -o run -- python3 <repo>/bench.py --pmc-driver",
               "cd /tmp && timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE --output-format csv "
               "-d <out>/pmc_write -o run -- python3 <repo>/bench.py --pmc-driver",
               "python bench.py --traffic-summary <out>/pmc_fetch/run_counter_collection.csv "
               "<out>/pmc_write/run_counter_collection.csv"]}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


def measured_traffic(args):
    """Bytes per finest FP32 sweep from the committed counter summary, or None
    when it is missing, was taken on other kernel sources or on another
    workload."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash() or t.get("workload") != traffic_workload(args):
        return None
    return t.get("traffic_bytes_per_sweep")


def kernel_of(B, args):
    if args.kernel == "const":
        return B.kernel(B.AMG_K_CONST)
    if args.kernel == "weighted":
        return B.kernel(B.AMG_K_WEIGHTED, wl=1.2, wr=0.8)
    return B.kernel(B.AMG_K_FRACTIONAL, alpha=args.alpha)


def run_form(B, torch, args, precision, b_dev, profile=False, inner=0):
    """Timed solves (graph-replayed V-cycles) or, with profile=True, the
    profiled pass: the same solves launched eagerly with HIP events around the
    finest-level FFT passes on the solve stream.  inner selects the outer
    iteration (0: the paper's stationary V-cycle iteration, 1: V-cycle-
    preconditioned CG)."""
    N = 2 ** args.logN
    flags = B.AMG_FLAG_PROFILE if profile else 0
    if not args.no_deep_fold:
        flags |= B.AMG_FLAG_DEEP_FOLD
    opts = B.amg_default_opts(precision=precision, flags=flags, max_iter=500, inner=inner)
    steps = args.prof_steps if profile else args.steps
    warmup = 1 if profile else args.warmup
    t0 = time.perf_counter()
    h = B.amg_setup(kernel_of(B, args), args.delta, N, opts)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    x = torch.zeros_like(b_dev)
    try:
        for _ in range(warmup):
            x.zero_()
            B.amg_solve(h, b_dev, x, args.tol)
        B.amg_profile_stats(h, reset=True)
        lat, iters = [], []
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(steps):
            x.zero_()  # each solve starts from x_0 = 0
            t1 = time.perf_counter()
            st, it, rel = B.amg_solve(h, b_dev, x, args.tol)
            lat.append(time.perf_counter() - t1)
            iters.append(it)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        prof = B.amg_profile_stats(h)
        # latency percentiles over at least LAT_SAMPLES solves: the timed ones
        # plus more of the same (these do not enter the throughput)
        for _ in range(max(0, LAT_SAMPLES - steps) if not profile else 0):
            x.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            B.amg_solve(h, b_dev, x, args.tol)
            lat.append(time.perf_counter() - t1)
        return dict(handle=None, x=x.clone(), setup_s=setup_s, wall_s=wall, lat=np.array(lat),
                    iters=iters, relres=rel, prof=prof)
    finally:
        B.amg_destroy(h)


def sweep_roofline(prof, n, prefix, p_bytes, sym):
    """Finest-level FFT matvec sweep: 3 passes timed from the event before
    pass 1 to the event after pass 3 (no events between the passes).
    Algorithmic bytes per sweep (one read
    and one write of each vector, one read of each spectrum and Cross
    vector): SPD 11 n p, general 16 n p."""
    launches, ms = prof.get(f"{prefix}_finest_sweep", (0, 0.0))
    if launches == 0:
        return None
    avg_s = ms / launches * 1e-3
    alg = (11 if sym else 16) * n * p_bytes
    ach = alg / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": f"{prefix} finest-level FFT matvec sweep (3 passes)",
            "alg_bytes_per_launch": alg, "avg_us": round(avg_s * 1e6, 2), "sweeps": launches,
            "passes_note": "per-pass durations: profiles/solve_N2e20_const_kernel_trace.txt"}


def summary(res, N):
    lat = res["lat"]
    steps = len(res["iters"])
    sps = steps / res["wall_s"]
    return {"solves_per_s": round(sps, 3), "unknowns_per_s": round(sps * (2 * N - 1), 1),
            "ms_per_solve": round(1e3 * res["wall_s"] / steps, 3),
            "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
            "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
            "latency_samples": int(len(lat)),
            "iters": int(np.median(res["iters"])), "final_relres": res["relres"],
            "setup_s": round(res["setup_s"], 3)}


BATCH_ALPHA = (0.2, 0.8)
BATCH_MAX_ITER = 4000


def batch_instances(count, seed=0):
    """The uneven batch: N = 2^K with K uniform on 10..16, delta uniform on
    [0.05, 0.3], constant or fractional kernel with even odds, alpha uniform
    on [0.2, 0.8], b ~ N(0, 1) per unknown.  The product-integration weights
    of the fractional kernel are finite only below alpha = 1/2; from 1/2 on
    the instances use the near-field rule (AMG_K_FRACTIONAL_NEAR, an
    extension: one symmetric quadratic on |t| <= h/2)."""
    rng = np.random.default_rng(seed)
    K = rng.integers(10, 17, size=count)
    delta = rng.uniform(0.05, 0.3, size=count)
    frac = rng.integers(0, 2, size=count)
    alpha = rng.uniform(*BATCH_ALPHA, size=count)
    out = []
    for i in range(count):
        N = 2 ** int(K[i])
        out.append(dict(N=N, delta=float(delta[i]), frac=bool(frac[i]), alpha=float(alpha[i]),
                        b=rng.standard_normal(2 * N - 1)))
    return out


def batch_kernel(B, d):
    """The instance's kernel: constant, fractional (alpha < 1/2) or the
    fractional kernel with the near-field rule (alpha >= 1/2)."""
    if not d["frac"]:
        return B.kernel(B.AMG_K_CONST)
    kind = B.AMG_K_FRACTIONAL if d["alpha"] < 0.5 else B.AMG_K_FRACTIONAL_NEAR
    return B.kernel(kind, alpha=d["alpha"])


def batch_workload_id(args):
    """What a counted-traffic measurement of the batch belongs to."""
    return {"instances": args.batch, "seed": 0, "tol": args.tol, "alpha": list(BATCH_ALPHA)}


def run_batch(B, torch, args):
    """All instances in one amg_solve_batch call (internal streams, graph-
    replayed V-cycles), mixed precision, V-cycle-preconditioned CG (every
    instance is symmetric positive definite), tol as the headline.  One
    untimed batch first (it captures each handle's V-cycle graph), then the
    timed one from x_0 = 0."""
    inst = batch_instances(args.batch)
    opts = B.amg_default_opts(precision=B.AMG_MIXED, inner=B.AMG_INNER_PCG,
                              max_iter=BATCH_MAX_ITER)
    hs, bs, xs = [], [], []
    t0 = time.perf_counter()
    try:
        for d in inst:
            hs.append(B.amg_setup(batch_kernel(B, d), d["delta"], d["N"], opts))
            bs.append(torch.from_numpy(d["b"]).cuda())
            xs.append(torch.zeros_like(bs[-1]))
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        tols = [args.tol] * len(hs)
        B.amg_solve_batch(hs, bs, xs, tols, allow=(B.AMG_OK, B.AMG_NOT_CONVERGED))
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, its, rels = B.amg_solve_batch(hs, bs, xs, tols,
                                          allow=(B.AMG_OK, B.AMG_NOT_CONVERGED))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
    finally:
        for h in hs:
            B.amg_destroy(h)
    unknowns = sum(2 * d["N"] - 1 for d in inst)
    # algorithmic bytes per CG iteration (symmetric, FP32 V-cycle + FP64
    # outer): V-cycle ~52 n p at p = 4, FP64 matvec 11 n * 8, CG vector work
    # (x, p, r, r_old, q, z: ~10 reads/writes of 2n doubles) ~160 n
    alg = sum(it * (52 * 4 + 88 + 160) * (d["N"] - 1) for it, d in zip(its, inst))
    return {"instances": len(inst), "unknowns": unknowns, "wall_s": round(wall, 4),
            "solves_per_s": round(len(inst) / wall, 2),
            "unknowns_per_s": round(unknowns / wall, 1),
            "iters_median": int(np.median(its)), "iters_max": int(max(its)),
            "max_relres": float(max(rels)), "not_converged": int(sum(r >= args.tol for r in rels)),
            "setup_s": round(setup_s, 2),
            "est_alg_bytes": alg, "est_alg_frac_of_hbm_peak": round(alg / wall / 1e9 / HBM_PEAK_GBS, 4),
            "counted_hbm_bytes": measured_batch_traffic(args),
            "counted_hbm_frac": (round(measured_batch_traffic(args) / wall / 1e9 / HBM_PEAK_GBS, 4)
                                 if measured_batch_traffic(args) else None),
            "near_field_instances": int(sum(d["frac"] and d["alpha"] >= 0.5 for d in inst)),
            "workload": "N=2^K, K~U{10..16}; delta~U[0.05,0.3]; const or fractional 50/50, "
                        "alpha~U[0.2,0.8] (alpha >= 1/2: AMG_K_FRACTIONAL_NEAR, the near-field "
                        "rule, an extension); b~N(0,1); seed 0; mixed, inner=PCG, "
                        f"tol={args.tol}, max_iter={BATCH_MAX_ITER}"}


def run_c2(B, torch, args):
    """The plain-method configurations: N = 2^14, 2^17, 2^20 intervals, delta in
    {0.05, 0.25}, the SPD constant kernel and the weighted 1.2/0.8 one,
    manufactured right-hand side, V-cycle to 2^5, tol as the headline, one
    solve at a time: FP64 and mixed solves/s (median of 5) and iterations; at
    2^14 and 2^17 the oracle times its own FP64 solve and evaluates the GPU
    solutions' residuals."""
    rows = []
    for logN in (14, 17, 20):
        N = 2 ** logN
        for delta in (0.05, 0.25):
            for kname in ("const", "weighted"):
                k = B.kernel(B.AMG_K_CONST) if kname == "const" else B.kernel(B.AMG_K_WEIGHTED, wl=1.2, wr=0.8)
                b = B.amg_manufactured_rhs(k, delta, N)
                bd = torch.from_numpy(b).cuda()
                row = {"N": N, "delta": delta, "kernel": kname}
                xs = {}
                for name, prec in (("fp64", B.AMG_FP64), ("mixed", B.AMG_MIXED)):
                    h = B.amg_setup(k, delta, N, B.amg_default_opts(precision=prec, max_iter=500))
                    try:
                        x = torch.zeros_like(bd)
                        B.amg_solve(h, bd, x, args.tol)
                        ts = []
                        for _ in range(5):
                            x.zero_()
                            torch.cuda.synchronize()
                            t0 = time.perf_counter()
                            st, it, rel = B.amg_solve(h, bd, x, args.tol)
                            ts.append(time.perf_counter() - t0)
                    finally:
                        B.amg_destroy(h)
                    xs[name] = x.cpu().numpy()
                    row[name] = {"solves_per_s": round(1.0 / float(np.median(ts)), 2), "iters": it,
                                 "relres": rel}
                if logN <= 17 and not args.no_cpu_baseline:
                    from oracle import discretize as D
                    from oracle import tpx
                    ok = (D.Kernel(D.CONST, delta) if kname == "const"
                          else D.Kernel(D.WEIGHTED, delta, wl=1.2, wr=0.8))
                    H = tpx.Hierarchy.build(tpx.from_stencil(ok, N), 5)
                    t0 = time.perf_counter()
                    _, ito, _ = tpx.solve(H, b, tol=args.tol, max_iter=500)
                    row["oracle"] = {"solves_per_s": round(1.0 / (time.perf_counter() - t0), 3),
                                     "iters": ito, "cores": tpx.WORKERS,
                                     "relres_of_gpu": {nm: float(np.linalg.norm(b - H.matvec(v)) / np.linalg.norm(b))
                                                       for nm, v in xs.items()}}
                rows.append(row)
    return rows


def timed_solves(B, torch, h, bd, tol, reps=5, x0=None):
    """Median wall time of `reps` solves (after one untimed), iterations and
    relres of the last."""
    x = torch.zeros_like(bd) if x0 is None else x0.clone()
    B.amg_solve(h, bd, x, tol, allow=(B.AMG_OK, B.AMG_NOT_CONVERGED))
    ts = []
    for _ in range(reps):
        if x0 is None:
            x.zero_()
        else:
            x.copy_(x0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, it, rel = B.amg_solve(h, bd, x, tol, allow=(B.AMG_OK, B.AMG_NOT_CONVERGED))
        ts.append(time.perf_counter() - t0)
    return {"ms_per_solve": round(1e3 * float(np.median(ts)), 3), "iters": it, "relres": rel,
            "converged": st == B.AMG_OK}


def run_extensions(B, torch, args):
    """The forms beyond the paper's stationary V-cycle on the bench size
    N = 2^20 (FP64 and mixed each): the standard (non-symmetric) collocation
    with non-zero volume data; one BDF4 step (shift 25/12, scale tau = h) of
    u = e^t x^2 (1-x)^2 from U^{k-1}; the weakly singular model (gamma = 0.5)
    in its BDF4 step system with a seeded random right-hand side; GMRES for
    the weighted kernel; and the stationary W-cycle iteration for the
    fractional kernel (alpha = 0.4, delta = 0.1) at N = 2^14 beside the
    V-cycle's."""
    N = 2 ** 20
    tol = args.tol
    out = {}
    rng = np.random.default_rng(7)
    forms = (("fp64", B.AMG_FP64), ("mixed", B.AMG_MIXED))
    # standard collocation, volume data g = (1+x)^6 on the interaction volume
    k = B.kernel(B.AMG_K_CONST, scheme=B.AMG_SCHEME_STANDARD)
    S = B.amg_volume_reach(k, 0.25, N)
    kk = np.arange(S + 1) / (2.0 * N)
    b = B.amg_manufactured_rhs(k, 0.25, N)
    b = B.amg_volume_rhs(k, 0.25, N, (1.0 - kk) ** 6, (2.0 + kk) ** 6, b)
    bd = torch.from_numpy(b).cuda()
    out["standard_volume_data"] = {}
    for name, prec in forms:
        h = B.amg_setup(k, 0.25, N, B.amg_default_opts(precision=prec))
        try:
            out["standard_volume_data"][name] = timed_solves(B, torch, h, bd, tol)
        finally:
            B.amg_destroy(h)
    # one BDF4 step of u = e^t x^2 (1-x)^2 (zero volume data), t_k = 4h
    kc = B.kernel(B.AMG_K_CONST)
    tau = 1.0 / N
    f = B.amg_manufactured_rhs(kc, 0.25, N)
    xs = np.concatenate([np.arange(1, N) / N, (np.arange(N) + 0.5) / N])
    u = xs * xs * (1 - xs) ** 2
    hist = [torch.from_numpy(np.exp(j * tau) * u).cuda() for j in (3, 2, 1, 0)]
    t4 = 4 * tau
    src = torch.from_numpy(tau * np.exp(t4) * (u + 2.0 * f)).cuda()  # kernel constant 3 delta^-3
    out["bdf4_step"] = {}
    for name, prec in forms:
        h = B.amg_setup(kc, 0.25, N, B.amg_default_opts(precision=prec, shift=25.0 / 12.0,
                                                       scale=2.0 * tau))
        try:
            # the step's initial residual b - M U^{k-1} is O(tau) of b: 1e-8 of it
            # is ~1e-14 of b (1e-10 would sit below what FP64 resolves at 2^20)
            tol_step = 1e-8
            ok = (B.AMG_OK, B.AMG_NOT_CONVERGED)
            xo = torch.empty_like(hist[0])
            B.amg_bdf4_step(h, hist, src, xo, tol_step, allow=ok)
            ts = []
            for _ in range(5):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, it, rel = B.amg_bdf4_step(h, hist, src, xo, tol_step, allow=ok)
                ts.append(time.perf_counter() - t0)
            err = float((xo.cpu().numpy() - np.exp(t4) * u).__abs__().max())
            out["bdf4_step"][name] = {"ms_per_step": round(1e3 * float(np.median(ts)), 3),
                                      "iters": it, "relres": rel, "tol": tol_step,
                                      "converged": st == B.AMG_OK, "max_err_vs_u": err}
        finally:
            B.amg_destroy(h)
    # the weakly singular model's BDF4 step system, random right-hand side
    kw = B.kernel(B.AMG_K_WEAKLY_SINGULAR, gamma=0.5)
    bw = torch.from_numpy(rng.standard_normal(2 * N - 1)).cuda()
    out["weakly_singular_step"] = {}
    for name, prec in forms:
        t0 = time.perf_counter()
        h = B.amg_setup(kw, 0.0, N, B.amg_default_opts(precision=prec, shift=25.0 / 12.0, scale=tau))
        setup = time.perf_counter() - t0
        try:
            r = timed_solves(B, torch, h, bw, tol)
            r["setup_s"] = round(setup, 2)
            out["weakly_singular_step"][name] = r
        finally:
            B.amg_destroy(h)
    # GMRES for the weighted kernel (manufactured right-hand side)
    kwt = B.kernel(B.AMG_K_WEIGHTED, wl=1.2, wr=0.8)
    bg = torch.from_numpy(B.amg_manufactured_rhs(kwt, 0.25, N)).cuda()
    out["gmres_weighted"] = {}
    for name, prec in forms:
        h = B.amg_setup(kwt, 0.25, N, B.amg_default_opts(precision=prec, inner=B.AMG_INNER_GMRES))
        try:
            out["gmres_weighted"][name] = timed_solves(B, torch, h, bg, tol)
        finally:
            B.amg_destroy(h)
    # W-cycle vs V-cycle, fractional kernel, N = 2^14 (FP64)
    kf = B.kernel(B.AMG_K_FRACTIONAL, alpha=0.4)
    Nf = 2 ** 14
    bf = torch.from_numpy(B.amg_manufactured_rhs(kf, 0.1, Nf)).cuda()
    out["wcycle_fractional_2e14"] = {}
    for name, cyc in (("W", 2), ("V", 1)):
        h = B.amg_setup(kf, 0.1, Nf, B.amg_default_opts(cycle=cyc, max_iter=2000))
        try:
            out["wcycle_fractional_2e14"][name] = timed_solves(B, torch, h, bf, tol, reps=2)
        finally:
            B.amg_destroy(h)
    return out


def representation_floor(tpx, T, b, x, seed=7):
    """||A dx|| / ||b|| for dx uniform in +-ulp(x_i)/2, by the oracle in
    extended precision: the relative residual that rounding the solution to
    FP64 alone leaves; no FP64 vector near x has a residual much below it."""
    g = np.random.default_rng(seed)
    dx = (g.random(x.size) - 0.5) * np.spacing(np.abs(x))
    Ad = tpx.residual_extended(T, np.zeros_like(x), dx)
    return float(np.sqrt(np.dot(Ad, Ad))) / np.linalg.norm(b)


def run_c3(B, torch, args):
    """The precision configuration: delta = 0.1, fractional kernel alpha =
    0.4, manufactured right-hand side, tol 1e-10, at N = 2^22 intervals
    (8,388,607 unknowns) and at N = 2^20.  Mixed form (FP32 V-cycle, FP64
    residual, update and coarsest solve) and FP64 form, both as V-cycle-
    preconditioned CG (the stationary iteration needs thousands of V-cycles
    here), with the split FP64 residual (near field in difference form, far
    field by FFT) so that the stopping test sees the true residual.  The
    oracle evaluates each solution's residual in extended precision and the
    FP64 representation floor of the solution: at 2^22 that floor is above
    1e-10, and the solve stops at it (status "fp64 floor")."""
    k = B.kernel(B.AMG_K_FRACTIONAL, alpha=0.4)
    out = {"workload": "delta=0.1, fractional alpha=0.4, manufactured u=x^2(1-x)^2, tol=1e-10, "
                       "inner=PCG, split FP64 residual (AMG_FLAG_ACCURATE_RESIDUAL)"}
    for logN in (22, 20):
        N = 2 ** logN
        b = B.amg_manufactured_rhs(k, 0.1, N)
        bd = torch.from_numpy(b).cuda()
        res, xs = {}, {}
        for name, prec in (("mixed", B.AMG_MIXED), ("fp64", B.AMG_FP64)):
            h = B.amg_setup(k, 0.1, N, B.amg_default_opts(
                precision=prec, inner=B.AMG_INNER_PCG, max_iter=1500,
                flags=B.AMG_FLAG_ACCURATE_RESIDUAL))
            try:
                x = torch.zeros_like(bd)
                B.amg_solve(h, bd, x, args.tol, allow=(B.AMG_OK, B.AMG_NOT_CONVERGED))  # warm-up
                x.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, it, rel = B.amg_solve(h, bd, x, args.tol, allow=(B.AMG_OK, B.AMG_NOT_CONVERGED))
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            finally:
                B.amg_destroy(h)
            xs[name] = x.cpu().numpy()
            res[name] = {"s_per_solve": round(dt, 4), "iters": it, "relres": rel,
                         "status": {B.AMG_OK: "ok", B.AMG_NOT_CONVERGED: "fp64 floor"}[st],
                         "unknowns_per_s": round((2 * N - 1) / dt, 1)}
        res["err_mixed_vs_fp64"] = float(np.abs(xs["mixed"] - xs["fp64"]).max()
                                         / np.abs(xs["fp64"]).max())
        if not args.no_cpu_baseline:
            from oracle import discretize as D
            from oracle import tpx
            T = tpx.from_stencil_rowsum(D.Kernel(D.FRACTIONAL, 0.1, alpha=0.4), N)
            for name in ("mixed", "fp64"):
                res[name]["relres_oracle_extended"] = float(tpx.relres_extended(T, b, xs[name]))
            res["fp64_representation_floor"] = representation_floor(tpx, T, b, xs["mixed"])
        out[f"N=2^{logN}"] = res
        print(f"# c3 N=2^{logN}: {res}", file=sys.stderr, flush=True)
    return out


def serve_requests(seconds, rate, seed=1):
    """The serving workload: Poisson arrivals at `rate` per second over
    `seconds`, N = 2^K with K uniform on 12..22, delta uniform on [0.02,
    0.3], constant or weighted (1.2 / 0.8, non-symmetric) kernel with even
    odds, tol 1e-8 or 1e-10 with even odds, b ~ N(0, 1) drawn on the device
    from a per-request seed."""
    g = np.random.default_rng(seed)
    out, t = [], 0.0
    while True:
        t += float(g.exponential(1.0 / rate))
        if t >= seconds:
            return out
        K = int(g.integers(12, 23))
        out.append(dict(t=t, K=K, N=2 ** K, delta=float(g.uniform(0.02, 0.3)),
                        weighted=bool(g.integers(0, 2)), tol=[1e-8, 1e-10][int(g.integers(0, 2))],
                        seed=int(g.integers(0, 2 ** 62))))


def run_serve(B, torch, args):
    """Open-loop serving: an arrival thread submits each request at its
    scheduled time (b drawn on the device); the main thread steps the server
    (one round over every request in flight per step, requests joining and
    leaving between rounds) and collects results.  Latency is from the
    scheduled arrival to the poll that returns the result.  Mixed precision,
    stationary V-cycle iteration (the weighted kernel is non-symmetric).  One
    untimed request per size first (module loads, twiddle tables)."""
    import threading
    reqs = serve_requests(args.serve_seconds, args.serve_rate)
    opts = B.amg_default_opts(precision=B.AMG_MIXED, max_iter=100)
    sv = B.amg_server_create(int(args.serve_budget_gb * 2 ** 30), workers=args.serve_workers)
    if args.serve_small_log2 > 0:
        B.amg_server_lanes(sv, 2 ** args.serve_small_log2, args.serve_small_rounds)
    lock = threading.Lock()
    live, done = {}, {}
    gen_stream = torch.cuda.Stream()  # the arrival side's stream for b and x

    def kern(r):
        return (B.kernel(B.AMG_K_WEIGHTED, wl=1.2, wr=0.8) if r["weighted"]
                else B.kernel(B.AMG_K_CONST))

    live_bytes = [0]
    shed = []

    def submit(i, r):
        vec_bytes = 2 * 8 * (2 * r["N"] - 1)
        with lock:
            if i >= 0 and live_bytes[0] + vec_bytes > args.serve_queue_gb * 2 ** 30:
                shed.append(i)  # the queue's vectors would pass their bound: load shedding
                return
            live_bytes[0] += vec_bytes
        gen = torch.Generator(device="cuda")
        gen.manual_seed(r["seed"])
        with torch.cuda.stream(gen_stream):
            b = torch.randn(2 * r["N"] - 1, generator=gen, device="cuda", dtype=torch.float64)
            x = torch.zeros_like(b)
        gen_stream.synchronize()  # the server reads b and x on its own stream
        with lock:
            rid = B.amg_server_submit(sv, kern(r), r["delta"], r["N"], b, x, r["tol"], opts)
            live[rid] = (i, b, x)

    def drain(deadline):
        while time.perf_counter() < deadline:
            with lock:
                if not live:
                    return True
            inflight, _ = B.amg_server_step(sv, args.serve_rounds)
            now = time.perf_counter()
            with lock:
                for res in B.amg_server_poll(sv):
                    i, bb, _ = live.pop(res[0])
                    live_bytes[0] -= 2 * bb.numel() * 8
                    done[i] = (now, res)
            if inflight == 0:
                time.sleep(2e-4)
        return False

    try:
        warm = [dict(N=2 ** K, K=K, delta=0.1, weighted=bool(K % 2), tol=1e-8, seed=K)
                for K in range(12, 23)]
        for i, r in enumerate(warm):
            submit(-1 - i, r)
        drain(time.perf_counter() + 120)
        done.clear()
        s0 = B.amg_server_stats(sv)
        t0 = time.perf_counter()

        def arrivals():
            for i, r in enumerate(reqs):
                wait = t0 + r["t"] - time.perf_counter()
                if wait > 0:
                    time.sleep(wait)
                submit(i, r)

        th = threading.Thread(target=arrivals)
        th.start()
        t_note = t0
        while th.is_alive():
            drain(time.perf_counter() + 0.05)
            if time.perf_counter() - t_note > 10:
                t_note = time.perf_counter()
                with lock:
                    print(f"# serve t={t_note - t0:.0f}s completed={len(done)} in flight={len(live)}",
                          file=sys.stderr, flush=True)
        th.join()
        finished = drain(t0 + args.serve_seconds + args.serve_drain_s)
        t_end = max((d[0] for d in done.values()), default=t0)
        s1 = B.amg_server_stats(sv)
    finally:
        B.amg_server_destroy(sv)
    lat = np.array([done[i][0] - t0 - reqs[i]["t"] for i in sorted(done)])
    ok = [i for i in done if done[i][1][1] == B.AMG_OK]
    unknowns = sum(2 * reqs[i]["N"] - 1 for i in done)
    wall = t_end - t0
    by_K = {}
    for K in range(12, 23):
        lk = [done[i][0] - t0 - reqs[i]["t"] for i in done if reqs[i]["K"] == K]
        if lk:
            by_K[f"2^{K}"] = {"n": len(lk), "p50_ms": round(1e3 * float(np.percentile(lk, 50)), 2),
                              "p99_ms": round(1e3 * float(np.percentile(lk, 99)), 2)}
    hits = s1["cache_hits"] - s0["cache_hits"]
    miss = s1["cache_misses"] - s0["cache_misses"]
    offered = sum(2 * r["N"] - 1 for r in reqs) / args.serve_seconds
    return {
        "workload": (f"Poisson arrivals {args.serve_rate}/s for {args.serve_seconds} s, seed 1; "
                     "N=2^K, K~U{12..22}; delta~U[0.02,0.3]; const or weighted (1.2/0.8) 50/50; "
                     "tol 1e-8 or 1e-10 50/50; b~N(0,1) on device; mixed, stationary V-cycle"),
        "requests": len(reqs), "completed": len(done), "shed": len(shed), "drained": finished,
        "ok": len(ok), "not_ok": len(done) - len(ok),
        "max_relres_over_tol": float(max((done[i][1][3] / reqs[i]["tol"] for i in ok), default=0.0)),
        "wall_s": round(wall, 3), "solves_per_s": round(len(done) / wall, 2),
        "unknowns_per_s": round(unknowns / wall, 1), "offered_unknowns_per_s": round(offered, 1),
        "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 2),
        "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 2),
        "max_ms": round(1e3 * float(lat.max()), 2), "latency_by_size": by_K,
        "iters_median": int(np.median([done[i][1][2] for i in done])),
        "rounds": s1["rounds"] - s0["rounds"],
        "cache_hits": hits, "cache_misses": miss,
        "cache_hit_rate": round(hits / max(hits + miss, 1), 4),
        "evictions": s1["evictions"] - s0["evictions"],
        "peak_reserved_gb": round(s1["peak_reserved_bytes"] / 2 ** 30, 2),
        "server_time_s": {k: round((s1[k + "_us"] - s0[k + "_us"]) / 1e6, 3)
                          for k in ("start", "rebuild", "rounds", "setup")},
        "plan_rebuilds": s1["rebuilds"] - s0["rebuilds"],
        "budget_gb": args.serve_budget_gb, "setup_workers": args.serve_workers,
        "lanes": ({"small_max_N": 2 ** args.serve_small_log2,
                   "small_rounds_per_round": args.serve_small_rounds}
                  if args.serve_small_log2 > 0 else None),
    }


def cpu_baseline(args, b, x_fp64, x_mixed):
    """The oracle (CPU FP64, scipy FFT) on the same workload: one full solve,
    hierarchy setup excluded, on the host's cores; also evaluates the GPU
    solutions' residuals and their error against the oracle's solution."""
    from oracle import discretize as D
    from oracle import tpx
    N = 2 ** args.logN
    ok = {"const": D.Kernel(D.CONST, args.delta),
          "weighted": D.Kernel(D.WEIGHTED, args.delta, wl=1.2, wr=0.8),
          "fractional": D.Kernel(D.FRACTIONAL, args.delta, alpha=args.alpha)}[args.kernel]
    t0 = time.perf_counter()
    H = tpx.Hierarchy.build(tpx.from_stencil(ok, N), 5)
    setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    xo, it, hist = tpx.solve(H, b, tol=args.tol, max_iter=500)
    dt = time.perf_counter() - t0
    nb = np.linalg.norm(b)
    out = {"value": round(1.0 / dt, 4), "unit": "solves/s", "cores": tpx.WORKERS,
           "kind": "oracle",
           "sample": f"1 full FP64 solve at N=2^{args.logN} ({it} V-cycles, {dt:.1f} s; "
                     f"hierarchy setup {setup:.1f} s excluded), same workload",
           "unknowns_per_s": round((2 * N - 1) / dt, 1), "iters": it}
    errs = {}
    for name, x in (("fp64", x_fp64), ("mixed", x_mixed)):
        errs[name] = {"relres_oracle": float(np.linalg.norm(b - H.matvec(x)) / nb),
                      "err_vs_oracle": float(np.abs(x - xo).max() / np.abs(xo).max())}
    return out, errs


def main():
    args = parse()
    if args.rocprof_summary:
        rocprof_summary(args.rocprof_summary)
        return
    if args.traffic_summary:
        traffic_summary(args.traffic_summary[0], args.traffic_summary[1], args.logN,
                        traffic_workload(args))
        return
    if args.pmc_driver:
        pmc_driver(args)
        return
    if args.pmc_batch_driver:
        pmc_batch_driver(args)
        return
    if args.batch_traffic_summary:
        batch_traffic_summary(args.batch_traffic_summary[0], args.batch_traffic_summary[1], args)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one MI355X; runs on more than one GPU are not "
              "supported (each solve is independent -- shard instances across GPUs instead)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2202_11288_amd import binding as B
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    tuned = None
    if not args.no_autotune:
        t0 = time.perf_counter()
        B.amg_autotune(13, 23)
        tuned = {"seconds": round(time.perf_counter() - t0, 3),
                 "note": "geometry (log2 row length, column tile) per level size 2^logL, chosen by "
                         "amg_autotune: FP32 + FP64 level matvec, median of 7, every candidate "
                         "checked against the default geometry's product",
                 "sizes": {f"2^{lg}": B.amg_plan_get(lg) for lg in range(13, 24)}}
        print(f"# autotune done: {tuned}", file=sys.stderr, flush=True)
    N = 2 ** args.logN
    b = B.amg_manufactured_rhs(kernel_of(B, args), args.delta, N)
    b_dev = torch.from_numpy(b).cuda()
    print(f"# bench: N=2^{args.logN} kernel={args.kernel} delta={args.delta} "
          f"steps={args.steps} warmup={args.warmup}", file=sys.stderr, flush=True)
    r64 = run_form(B, torch, args, B.AMG_FP64, b_dev)
    print(f"# fp64 done: {summary(r64, N)}", file=sys.stderr, flush=True)
    rmx = run_form(B, torch, args, B.AMG_MIXED, b_dev)
    print(f"# mixed done: {summary(rmx, N)}", file=sys.stderr, flush=True)
    s64, smx = summary(r64, N), summary(rmx, N)
    sym = args.kernel != "weighted"
    krylov = None
    if sym and not args.no_pcg:
        k64 = summary(run_form(B, torch, args, B.AMG_FP64, b_dev, inner=B.AMG_INNER_PCG), N)
        kmx = summary(run_form(B, torch, args, B.AMG_MIXED, b_dev, inner=B.AMG_INNER_PCG), N)
        print(f"# pcg done: fp64 {k64} mixed {kmx}", file=sys.stderr, flush=True)
        krylov = {"note": "V-cycle-preconditioned CG (inner = AMG_INNER_PCG): same V-cycle, "
                          "Krylov outer iteration; not the paper's stationary iteration",
                  "mixed": kmx, "fp64": k64}
    # the request loop and the batch first, while the process holds no
    # leftovers of the host-heavy legs (their set-up threads share the host
    # with it; measured: p50 25 vs 38 ms when it ran after them)
    serve = None
    if args.serve_seconds > 0:
        serve = run_serve(B, torch, args)
        print(f"# serve done: {serve}", file=sys.stderr, flush=True)
    batch = None
    if args.batch > 0:
        batch = run_batch(B, torch, args)
        print(f"# batch done: {batch}", file=sys.stderr, flush=True)
    c2 = None
    if not args.no_c2:
        c2 = run_c2(B, torch, args)
        print(f"# c2 done: {c2}", file=sys.stderr, flush=True)
    ext = None
    if not args.no_ext:
        ext = run_extensions(B, torch, args)
        print(f"# extensions done: {ext}", file=sys.stderr, flush=True)
    c3 = None
    if not args.no_c3:
        c3 = run_c3(B, torch, args)
        print(f"# c3 done: {c3}", file=sys.stderr, flush=True)
    n = N - 1
    roof = roof64 = roof32 = None
    if args.prof_steps > 0:
        p64 = run_form(B, torch, args, B.AMG_FP64, b_dev, profile=True)["prof"]
        pmx = run_form(B, torch, args, B.AMG_MIXED, b_dev, profile=True)["prof"]
        print("# profiled passes done", file=sys.stderr, flush=True)
        roof64 = sweep_roofline(p64, n, "fp64", 8, sym)
        roof32 = sweep_roofline(pmx, n, "fp32", 4, sym)
        # dominant kernel of the headline (mixed) form
        t32 = pmx.get("fp32_finest_sweep", (0, 0.0))[1]
        t64 = pmx.get("fp64_finest_sweep", (0, 0.0))[1]
        roof = roof32 if t32 >= t64 else sweep_roofline(pmx, n, "fp64", 8, sym)
        if roof is roof32 and roof32 is not None:
            tb = measured_traffic(args)
            roof32["traffic"] = tb
            if tb:
                rate = tb / (roof32["avg_us"] * 1e-6) / 1e9
                roof32["traffic_gbs"] = round(rate, 1)
                roof32["traffic_frac"] = round(rate / HBM_PEAK_GBS, 4)
                roof32["traffic_note"] = ("HBM bytes per sweep from rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                          "scaled by a plain copy of known size (profiles/); "
                                          "traffic_gbs = those bytes over the sweep's time")
    cpu, errs = (None, None)
    if not args.no_cpu_baseline:
        cpu, errs = cpu_baseline(args, b, r64["x"].cpu().numpy(), rmx["x"].cpu().numpy())
    out = {
        "metric": "solves/s & unknowns/s at N=2^20, FP32+refine vs plain FP64; p50/p99 latency",
        "value": smx["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": smx["ms_per_solve"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 V-cycle + f64 refinement",
        "data": "synthetic",
        "config": {"workload": f"manufactured u=x^2(1-x)^2, {args.kernel} kernel, delta={args.delta}, "
                               f"N=2^{args.logN} intervals ({2 * N - 1} unknowns), tol={args.tol}, "
                               "V-cycle to 2^5, omega=2/3, m1=m2=1"
                               + ("" if args.no_deep_fold else
                                  ", levels <= 2^11 as one folded dense product (AMG_FLAG_DEEP_FOLD)"),
                   "N": N, "unknowns": 2 * N - 1, "delta": args.delta, "kernel": args.kernel,
                   "tol": args.tol},
        "unknowns_per_s": smx["unknowns_per_s"],
        "mixed": smx, "fp64": s64,
        "speedup_mixed_vs_fp64": round(smx["solves_per_s"] / s64["solves_per_s"], 3),
        "pcg": krylov,
        "batch": batch,
        "serving": serve,
        "autotune": tuned,
        "plain_configs": c2,
        "extensions": ext,
        "precision_config": c3,
        "roofline": roof, "roofline_fp64_form": roof64, "roofline_fp32_sweep": roof32,
        "roofline_source": (f"HIP events around the finest-level FFT passes on the solve stream, "
                            f"{args.prof_steps} profiled solves per form launched eagerly "
                            "(the timed solves replay the captured V-cycle graph)"),
        "cpu_baseline": cpu, "oracle_check": errs,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
