#!/usr/bin/env python3
"""Benchmark of the FFT nonlinear-stencil American option pricer on one MI355X.

A step prices one batch of seeded synthetic options (default: 64 binomial
American calls at T = 2^20, the large size of the binomial FFT-vs-plain
workload) through the C ABI.  Prints one JSON line:

  value        whole-job equivalent lattice cells per second, sum(T^2) / time
  roofline     the solver kernel's algorithmic HBM bytes per launch (sum over
               FFT correlations of 8 (n_in + n_out) bytes, plus the directly
               computed expiry-adjacent row) over its average launch time,
               against the 8 TB/s HBM3E peak; band_fp64 gives the band
               stencil's FP64 rate against the 78.6 TFLOP/s vector peak
  accuracy     per-option error against stored oracle prices of the same
               options; all_ok requires every checked option within the FP64
               tolerance
  plain_gpu    the plain Theta(T^2) GPU stencil on the same batch (one step)
               and the FFT path's speed-up over it
  extra        the other seeded workloads (trinomial mixed precision 2^20,
               BSM 2^18 FP64 and mixed, European 2^20), each with its
               throughput and per-option errors, and the Gaussian
               approximations of the European binomial call with their error
               against the exact lattice value
  serve        the serving mix: capacity, p50/p99 latency at 0.7 capacity,
               and the served batches' algorithmic bytes against HBM peak
  cpu_baseline the CPU oracle (plain Theta(T^2) induction) on a bounded
               sample, one option per host thread
  cpu_fft_method the same FFT method on host cores (OpenMP) at the paper's
               parameter point, by thread count

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--log2T 20]
                       [--options 64] [--option-type binomial|trinomial|bsm]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "equiv. lattice cells/s (T^2/t) at ≤1e-6 rel err vs FP64; serve p50/p99 latency"
HBM_PEAK_GBS = 8000.0
FP64_VEC_PEAK_TFLOPS = 78.6
TYPES = {"binomial": 0, "trinomial": 1, "bsm": 2}
CONFIG_ID = {0: 2, 1: 3, 2: 4}  # seeded workload ids of the three option types
GOLDEN_NAME = {0: "binomial", 1: "trinomial", 2: "bsm"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("aop_solver.hip", "aop_internal.h")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "solve_kernel_binomial_T2p20_64opt_hbm_traffic.md")


def kernel_sources_sha256() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2303_02317_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per solve_kernel launch from the committed counter summary.

    The summary lists `key: value` lines; its figure is used only for the
    workload it was measured on and only while the kernel sources hash to the
    value recorded with it (null otherwise: the counters describe other code).
    """
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None, "no counter summary"
    kv = {}
    for line in open(TRAFFIC_SUMMARY):
        line = line.strip().lstrip("-* ").strip()
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip().strip("`")] = v.strip().strip("`")
    if kv.get("workload") != workload:
        return None, "counters were taken on another workload"
    if kv.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None, "kernel changed since the counters were taken"
    try:
        return float(kv["traffic_bytes_per_launch"]), "rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated"
    except (KeyError, ValueError):
        return None, "summary has no traffic figure"


def golden_prices(model: int, log2T: int, european: bool = False):
    """Stored oracle prices of the seeded batch (tests/golden/make_golden.py), or None."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_%s%s_c%d_t%d.json" % (
        "european_" if european else "", GOLDEN_NAME[model], CONFIG_ID[model], log2T))
    if not os.path.exists(path):
        return None
    doc = json.load(open(path))
    return [r["price"] for r in doc["options"]]


def accuracy_of(prices, ref, opts, mixed: bool = False):
    """Errors against stored oracle prices (relative for prices >= 1e-3 K, absolute
    in units of K below), with the per-option lists and the verdict against the
    FP64 (1e-9 / 1e-13 K) or mixed-precision (1e-6 / 1e-9 K) tolerance."""
    if ref is None:
        return None
    rel_tol, abs_tol = (1e-6, 1e-9) if mixed else (1e-9, 1e-13)
    k = min(len(ref), len(opts))
    big = [i for i in range(k) if abs(ref[i]) >= 1e-3 * opts[i]["K"]]
    small = [i for i in range(k) if abs(ref[i]) < 1e-3 * opts[i]["K"]]
    rel = [abs(prices[i] - ref[i]) / abs(ref[i]) for i in big]
    ab = [abs(prices[i] - ref[i]) / opts[i]["K"] for i in small]
    finite = all(math.isfinite(float(prices[i])) for i in range(k))
    within = finite and all(r <= rel_tol for r in rel) and all(a <= abs_tol for a in ab)
    return {"n_checked": k, "n_options": len(opts), "n_rel": len(big),
            "max_rel_err": max(rel) if rel else None, "n_small": len(small),
            "max_abs_err_over_K_small": max(ab) if ab else None,
            "per_option_abs_err": [abs(float(prices[i]) - ref[i]) for i in range(k)],
            "per_option_rel_err": [abs(float(prices[i]) - ref[i]) / max(abs(ref[i]), 1e-300) for i in range(k)],
            "tolerance": {"rel": rel_tol, "abs_over_K": abs_tol},
            "within_tolerance": within, "reference": "CPU oracle (FP64), stored"}


def timed_batch(ctx, opts, precision, steps, warmup):
    """Warm up, then time `steps` launches of one batch with HIP events on its stream."""
    import torch

    from paper_2303_02317_amd import binding

    stream = torch.cuda.current_stream()
    ws = torch.empty(binding.workspace_bytes(opts, precision), dtype=torch.uint8, device="cuda")
    L = None
    for _ in range(warmup):
        L = binding.launch_batch(ctx, opts, precision=precision, workspace=ws)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        evs[k][0].record(stream)
        L = binding.launch_batch(ctx, opts, precision=precision, workspace=ws)
        evs[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return L, wall, [a.elapsed_time(b) for a, b in evs]


def extra_leg(ctx, name, model, log2T, precision, european=False, steps=2, warmup=1, n=64):
    """One more seeded workload: throughput and per-option error against stored oracle prices."""
    import numpy as np

    from paper_2303_02317_amd import autotune, binding, inputs

    opts = inputs.batch(CONFIG_ID[model], log2T, n, model)
    if european:
        opts = [dict(o, european=True) for o in opts]
    autotune.apply(ctx, model, 1 << log2T, precision)
    log("%s: %s T=2^%d %d options %s%s" % (name, GOLDEN_NAME[model], log2T, n, "mixed" if precision else "fp64",
                                          " european" if european else ""))
    L, wall, ms = timed_batch(ctx, opts, precision, steps, warmup)
    prices = L.price.cpu().numpy()
    cells = sum(float(o["T"]) ** 2 for o in opts)
    acc = accuracy_of(prices, golden_prices(model, log2T, european), opts, mixed=precision == 1)
    ok = bool(np.all(L.status == 0) and np.all(np.isfinite(prices))) and (acc is None or acc["within_tolerance"])
    return {"workload": "%s American %s%s, T=2^%d, %d seeded options, %s" % (
                GOLDEN_NAME[model], "put" if model == 2 else "call", " (European exercise)" if european else "",
                log2T, n, "split-FP32 correlations, FP64 band/boundary/root" if precision else "FP64"),
            "value": cells * steps / wall, "unit": "cells/s", "ms_per_step": wall / steps * 1e3,
            "launch_ms": ms, "precision": "mixed" if precision else "fp64", "accuracy": acc, "all_ok": ok}


def cpu_baseline(opts_full, model, log2T, budget_s=20.0):
    """Time the CPU oracle on a bounded sample of the workload's option batch."""
    import oracle
    from paper_2303_02317_amd import inputs

    # the GPU machine gives one GPU a share of 16 host cores, whatever the machine reports
    cores = min(len(os.sched_getaffinity(0)), 16)
    # Sample: the first options of the same seeded batch, at a T whose Theta(T^2)
    # oracle cost per option is a few seconds (the oracle's T^2/s rate does not
    # depend on T); 4 options per thread.
    sT = min(log2T, 17 if model == 0 else 16)
    sample = inputs.batch(CONFIG_ID[model], sT, 4 * cores, model)
    oracle.build()
    t0 = time.perf_counter()
    oracle.price_many(sample, threads=cores)
    dt = time.perf_counter() - t0
    cells = sum(float(o["T"]) ** 2 for o in sample)
    return {"value": cells / dt, "unit": "cells/s", "cores": cores, "kind": "oracle",
            "seconds": round(dt, 3),
            "sample": "first %d options of the same seeded batch (config id %d) at T=2^%d on %d host threads "
                      "(4 options each), plain FP64 backward induction" % (len(sample), CONFIG_ID[model], sT, cores)}


def serve_bench(ctx, n_req: int, load: float = 0.7, max_inflight: int = 4, max_batch: int = 64):
    """Serving mix: closed-loop capacity, then an open loop of Poisson arrivals at load x capacity."""
    import numpy as np

    from paper_2303_02317_amd import binding, inputs

    opts = inputs.serving_mix(n_req)
    cells = np.array([float(o["T"]) ** 2 for o in opts])
    from paper_2303_02317_amd import autotune

    # per size class schedules from the committed autotuner table
    cfg = dict(hbm_budget=48 << 30, max_inflight=max_inflight, max_batch=max_batch, tunings=autotune.server_table())

    def collect(srv, n, got, t_end=None):
        while len(got) < n:
            for r in srv.poll(8192, 2000):
                got[r["id"]] = r
            if t_end is not None and time.perf_counter() > t_end:
                raise RuntimeError("serving run stalled: %s" % srv.stats())

    # closed loop: everything queued at once
    srv = binding.Server(ctx, **cfg)
    t0 = time.perf_counter()
    srv.submit(opts, list(range(len(opts))))
    got = {}
    collect(srv, len(opts), got, t0 + 600)
    wall = time.perf_counter() - t0
    st_closed = srv.stats()
    srv.close()
    cap = len(opts) / wall
    log("serve closed loop: %d requests in %.2f s (%.0f options/s)" % (len(opts), wall, cap))
    # open loop at `load` of the capacity
    rate = load * cap
    arr = inputs.poisson_arrivals(len(opts), rate)
    srv = binding.Server(ctx, **cfg)
    got2 = {}
    t0 = time.perf_counter()
    k = 0
    while k < len(opts):
        now = time.perf_counter() - t0
        j = k
        while j < len(opts) and arr[j] <= now:
            j += 1
        if j > k:
            srv.submit(opts[k:j], list(range(k, j)))
            k = j
        for r in srv.poll(8192, 0):
            got2[r["id"]] = r
        time.sleep(0.0002)
    collect(srv, len(opts), got2, time.perf_counter() + 600)
    wall2 = time.perf_counter() - t0
    st_open = srv.stats()
    srv.close()
    lat = np.array([got2[i]["latency_s"] for i in range(len(opts))])
    que = np.array([got2[i]["queue_s"] for i in range(len(opts))])
    ok = all(got[i]["status"] == 0 for i in got) and all(got2[i]["status"] == 0 for i in got2)
    same = all(got[i]["price"] == got2[i]["price"] for i in range(len(opts)))
    log("serve open loop at %.0f/s: p50 %.1f ms p99 %.1f ms" % (rate, 1e3 * np.percentile(lat, 50),
                                                              1e3 * np.percentile(lat, 99)))
    return {"requests": len(opts), "mix": "model uniform {binomial call, trinomial call, BSM put}, "
                                         "T = round(2^U[10,20]), parameters as the binomial batch, seed [5, 0]",
            "closed_loop": {"seconds": wall, "options_per_s": cap, "cells_per_s": float(cells.sum()) / wall,
                            "batches": st_closed["batches"], "peak_hbm_bytes": st_closed["peak_bytes"]},
            "open_loop": {"arrival_rate_per_s": rate, "load": load, "seconds": wall2,
                          "options_per_s": len(opts) / wall2, "cells_per_s": float(cells.sum()) / wall2,
                          "latency_p50_ms": 1e3 * float(np.percentile(lat, 50)),
                          "latency_p99_ms": 1e3 * float(np.percentile(lat, 99)),
                          "queue_p50_ms": 1e3 * float(np.percentile(que, 50)),
                          "batches": st_open["batches"], "peak_hbm_bytes": st_open["peak_bytes"]},
            "roofline": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                         "achieved": st_closed["alg_bytes"] / wall / 1e9,
                         "frac": st_closed["alg_bytes"] / wall / 1e9 / HBM_PEAK_GBS,
                         "alg_bytes": st_closed["alg_bytes"],
                         "note": "closed loop: algorithmic bytes of the served batches over the wall time"},
            "config": dict({k: v for k, v in cfg.items() if k != "tunings"}, precision="fp64",
                           tuned_classes=len(cfg["tunings"])),
            "all_ok": ok, "same_prices_both_runs": same}


def approx_leg(ctx, n=64, log2T=20):
    """Gaussian approximations of the European binomial call: time per batch
    and error against the exact lattice value (stored oracle sums)."""
    import torch

    from paper_2303_02317_amd import binding, inputs

    opts = inputs.batch(CONFIG_ID[0], log2T, n, 0)
    ref = golden_prices(0, log2T, european=True)
    out = {}
    for method, name in ((0, "window_6sd_O(sqrt T)"), (1, "sum_O(T)"), (2, "erf_O(1)")):
        binding.european_approx(ctx, opts, method)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p, st = binding.european_approx(ctx, opts, method)
        dt = time.perf_counter() - t0
        rel = [abs(p[i] - ref[i]) / ref[i] for i in range(min(len(ref), n)) if ref[i] >= 1e-3 * opts[i]["K"]] \
            if ref else []
        out[name] = {"ms_per_batch": dt * 1e3, "max_rel_err_vs_exact_lattice": max(rel) if rel else None,
                     "all_status_ok": bool((st == 0).all())}
    return {"workload": "European binomial call, T=2^%d, %d seeded options (approximations of the lattice value)"
                        % (log2T, n), "methods": out}


def cpu_method_leg():
    """The method itself on host cores (libaop_cpu, OpenMP tasks) at the paper's
    parameter point (Sec. 5), binomial call, T = 2^15 and 2^19, by thread
    count: the shape of the paper's scalability table on this machine's cores."""
    from paper_2303_02317_amd import cpu, inputs

    P = inputs.PAPER_POINT
    cores = min(len(os.sched_getaffinity(0)), 16)
    out = {"workload": "binomial American call at the paper's parameter point (S=127.62, K=130, R=0.00163, "
                       "Y=0.0163, V=0.2, E=252/365 y), one option", "cores_available": cores, "runs": []}
    for log2T, threads, reps in ((15, (1, 2, 4, 8, 16), 3), (19, (1, 16), 1)):
        o = inputs.option(0, P["S0"], P["K"], P["r"], P["q"], P["sigma"], P["expiry"], 1 << log2T)
        for th in threads:
            if th > cores:
                continue
            best = None
            for _ in range(reps):
                t0 = time.perf_counter()
                pr, st, _ = cpu.price_batch([o], threads=th, base=8)
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
            out["runs"].append({"T": 1 << log2T, "threads": th, "ms": best * 1e3, "price": float(pr[0]),
                                "cells_per_s": float(1 << log2T) ** 2 / best})
    log("cpu method: %s" % ["T=%d p=%d %.1f ms" % (r["T"], r["threads"], r["ms"]) for r in out["runs"]])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--log2T", type=int, default=20)
    ap.add_argument("--options", type=int, default=64)
    ap.add_argument("--option-type", choices=sorted(TYPES), default="binomial")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=4096,
                    help="requests of the serving mix timed after the batch (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB device buffer twice (reference kernel for HBM byte counters)")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip timing the plain Theta(T^2) GPU stencil on the same batch (one step)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (trinomial mixed 2^20, BSM 2^18 FP64 and mixed, European 2^20)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the pricer shards by option across GPUs with no collectives, "
              "and this build measures the one-GPU share (got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2303_02317_amd import binding, inputs

    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        x = torch.full((nbytes // 8,), 1.0, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(2):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 2}), flush=True)
        return

    model = TYPES[args.option_type]
    opts = inputs.batch(CONFIG_ID[model], args.log2T, args.options, model)
    n = len(opts)
    cells = sum(float(o["T"]) ** 2 for o in opts)
    log("bench: %s, T=2^%d, %d options, steps=%d warmup=%d" % (args.option_type, args.log2T, n, args.steps,
                                                               args.warmup))
    ctx = binding.Context(0)
    from paper_2303_02317_amd import autotune

    autotune.apply(ctx, model, 1 << args.log2T, 0)  # the tuned schedule of this size class, if any
    stream = torch.cuda.current_stream()
    ws = torch.empty(binding.workspace_bytes(opts), dtype=torch.uint8, device="cuda")
    L = None
    for w in range(args.warmup):
        L = binding.launch_batch(ctx, opts, workspace=ws)
        torch.cuda.synchronize()
        log("warmup step %d done" % w)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record(stream)
        L = binding.launch_batch(ctx, opts, workspace=ws)
        evs[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [a.elapsed_time(b) for a, b in evs]
    log("timed %d steps: %.3f s wall, launches %s ms" % (args.steps, wall, ["%.2f" % x for x in launch_ms]))

    prices = L.price.cpu().numpy()
    status = L.status
    st = binding.batch_stats(L, n)
    F = {f: i for i, f in enumerate(binding.STATS_FIELDS)}
    alg_bytes = 8.0 * float(st[:, F["conv_in"]].sum() + st[:, F["conv_out"]].sum() + st[:, F["direct_cells"]].sum())
    band_rows = float(st[:, F["band_rows"]].sum())
    band_flops = band_rows * 64 * (3.0 if model == 0 else 5.0)  # per lane: 1 mul + 1 fma (+1 fma trinomial/BSM)
    avg_s = float(np.mean(launch_ms)) / 1e3
    achieved = alg_bytes / avg_s / 1e9

    # Relative error is reported for prices >= 1e-3 K; below that the FFT's
    # normwise error makes it meaningless, and the absolute error in units of
    # K is reported instead (tolerances 1e-9 relative / 1e-13 K for FP64).
    accuracy = accuracy_of(prices, golden_prices(model, args.log2T), opts)
    ok = bool(np.all(status == 0) and np.all(np.isfinite(prices))) and bool(accuracy and accuracy["within_tolerance"])
    workload = "%s American %s, FFT nonlinear stencil, T=2^%d, %d seeded options" % (
        args.option_type, "put" if model == 2 else "call", args.log2T, n)
    traffic, traffic_src = measured_traffic(workload)

    line = {
        "metric": METRIC,
        "value": cells * args.steps / wall,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload,
                   "option_type": args.option_type, "T": 1 << args.log2T, "options": n,
                   "seed": [CONFIG_ID[model], args.log2T], "precision": "fp64", "gpus": 1},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_source": traffic_src,
                     "kernel": "solve_kernel", "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": avg_s * 1e3},
        "band_fp64": {"achieved": band_flops / avg_s / 1e12, "peak": FP64_VEC_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": band_flops / avg_s / 1e12 / FP64_VEC_PEAK_TFLOPS, "band_rows_per_launch": band_rows},
        "work": {f: int(st[:, i].sum()) for f, i in F.items()
                 if f not in ("max_depth", "reserved") and not f.startswith("cyc_")},
        "accuracy": accuracy,
        "all_ok": ok,
    }
    line["work"]["max_depth"] = int(st[:, F["max_depth"]].max())
    tot = float(st[:, F["cyc_total"]].sum()) or 1.0
    line["phases"] = {k: float(st[:, F["cyc_" + k]].sum()) / tot for k in ("band", "tiles", "wait", "rows")}
    line["phases"]["cycles_per_option"] = tot / max(n, 1)
    pool = binding.pool_stats(L, n)
    busy = pool["helper_busy"] + pool["helper_idle"]
    line["pool"] = dict(pool, helper_busy_frac=(pool["helper_busy"] / busy) if busy else None,
                        tuning=ctx.tuning())
    if not args.no_plain:
        log("plain O(T^2) GPU stencil on the same batch ...")
        wsp = torch.empty(binding.plain_workspace_bytes(opts), dtype=torch.uint8, device="cuda")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        e0.record(stream)
        P = binding.launch_plain(ctx, opts, workspace=wsp)
        e1.record(stream)
        torch.cuda.synchronize()
        pw = time.perf_counter() - t1
        pp = P.price.cpu().numpy()
        agree = float(np.max(np.abs(pp - prices) / np.maximum(np.abs(pp), 1e-3 * np.array([o["K"] for o in opts]))))
        line["plain_gpu"] = {"value": cells / pw, "unit": "cells/s", "ms": pw * 1e3, "event_ms": e0.elapsed_time(e1),
                             "speedup_fft_vs_plain": pw / (wall / args.steps), "max_rel_diff_vs_fft": agree}
    if not args.no_extra:
        line["extra"] = {
            "trinomial_mixed_T2p20": extra_leg(ctx, "config 3", 1, 20, 1),
            "bsm_fp64_T2p18": extra_leg(ctx, "config 4", 2, 18, 0),
            "bsm_mixed_T2p18": extra_leg(ctx, "config 4", 2, 18, 1),
            "binomial_european_T2p20": extra_leg(ctx, "European", 0, 20, 0, european=True),
            "trinomial_european_T2p20": extra_leg(ctx, "European", 1, 20, 0, european=True),
            "binomial_european_gauss_approx_T2p20": approx_leg(ctx),
        }
        autotune.apply(ctx, model, 1 << args.log2T, 0)
    if args.serve_requests > 0:
        log("serving mix ...")
        line["serve"] = serve_bench(ctx, args.serve_requests)
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        line["cpu_baseline"] = cpu_baseline(opts, model, args.log2T)
        line["cpu_fft_method"] = cpu_method_leg()
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
