"""Autotuner of the FFT path's launch schedule.

The tunables are those of ``aop_tuning``: which correlations are handed to
the work pool (``pub_min_lg``: the smallest published transform, 2^lg points),
which short correlations are stepped directly instead of transformed
(``direct_max_h``, ``direct_max_n``), the largest FP64 transform held whole in
LDS (``lds_max_lg``), the radix of the LDS butterfly passes (``radix_lg``) and
the persistent grid size.  The pool settings change no result (each option's
arithmetic is the same whoever computes a tile); the other knobs choose
between exact evaluations of the same linear map, so they move prices by
rounding only.  A candidate is accepted if its prices agree with the first
candidate's within 1e-9 (relative, or 1e-13 K below 1e-3 K, the FP64 parity
bar).

For each size class (model, ceil(log2 T), precision) the tuner times every
candidate schedule on a seeded batch of that class (median of four launches)
and keeps the fastest, unless it beats the first (library default) schedule by
no more than ``NOISE``; the
table is stored as JSON per device architecture and applied per class:
``apply(ctx, model, T, precision)`` sets a context's tuning before a batch
launch, and ``server_table`` gives the per-class table a server takes.

Usage on a GPU machine:  python -m paper_2303_02317_amd.autotune [--classes ...]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning_gfx950.json")

# FFT schedule candidates: publication threshold, direct-stepping limits,
# the largest FP64 transform held whole in LDS (2^11 or 2^12 points; longer
# correlations use four-step transforms of 2048-point rows) and the radix of
# the LDS butterfly passes (2^3 or 2^2).
CANDIDATES = [
    dict(pub_min_lg=13, direct_max_h=320, direct_max_n=2048),
    dict(pub_min_lg=12, direct_max_h=320, direct_max_n=2048),
    dict(pub_min_lg=14, direct_max_h=320, direct_max_n=2048),
    dict(pub_min_lg=15, direct_max_h=320, direct_max_n=2048),
    dict(pub_min_lg=16, direct_max_h=320, direct_max_n=2048),
    dict(pub_min_lg=20, direct_max_h=320, direct_max_n=2048),
    dict(pub_min_lg=13, direct_max_h=448, direct_max_n=2048),
    dict(pub_min_lg=14, direct_max_h=448, direct_max_n=2048),
    dict(pub_min_lg=11, direct_max_h=320, direct_max_n=2048),
    dict(pub_min_lg=12, direct_max_h=448, direct_max_n=2048),
    dict(pub_min_lg=11, direct_max_h=448, direct_max_n=2048),
    dict(pub_min_lg=10, direct_max_h=320, direct_max_n=2048),
    dict(pub_min_lg=10, direct_max_h=448, direct_max_n=2048),
    dict(pub_min_lg=11, direct_max_h=448, direct_max_n=2048, lds_max_lg=11),
    dict(pub_min_lg=12, direct_max_h=448, direct_max_n=2048, lds_max_lg=11),
    dict(pub_min_lg=11, direct_max_h=448, direct_max_n=2048, radix_lg=2),
    dict(pub_min_lg=12, direct_max_h=448, direct_max_n=2048, radix_lg=2),
    dict(pub_min_lg=11, direct_max_h=448, direct_max_n=2048, lds_max_lg=11, radix_lg=2),
]
#: Keys every stored schedule carries (missing ones take the library's defaults).
SCHEDULE_KEYS = ["pub_min_lg", "direct_max_h", "direct_max_n", "lds_max_lg", "radix_lg"]
SCHEDULE_DEFAULTS = dict(lds_max_lg=12, radix_lg=3)
#: A candidate replaces the first (library default) schedule only when its
#: median launch is shorter by more than this fraction: launches of one
#: schedule vary by about 1 % between repetitions.
NOISE = 0.015

#: Size classes timed by default: the benchmark workloads' (model, log2 T).
DEFAULT_CLASSES = [(0, 14), (0, 17), (0, 20), (1, 16), (1, 18), (1, 20), (2, 16), (2, 18)]
CONFIG_ID = {0: 2, 1: 3, 2: 4}


def class_key(model: int, lg: int, precision: int) -> str:
    return "m%d_lg%d_p%d" % (model, lg, precision)


def ceil_log2(T: int) -> int:
    return max(0, math.ceil(math.log2(max(1, T))))


def load_cache(path: str = CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def lookup(table: dict, model: int, T: int, precision: int = 0):
    """Best schedule for the class of (model, T, precision): the nearest tuned log2 T of that model."""
    lg = ceil_log2(T)
    best, dist = None, None
    for key, rec in table.get("classes", {}).items():
        m, l, p = rec["model"], rec["lg"], rec["precision"]
        if m != model:
            continue
        d = abs(l - lg) + (0 if p == precision else 0.5)
        if dist is None or d < dist:
            best, dist = rec["best"], d
    return best


def apply(ctx, model: int, T: int, precision: int = 0, table: dict | None = None) -> dict | None:
    """Set ctx's tuning to the tuned schedule of the class (no change if none is known)."""
    t = lookup(table if table is not None else load_cache(), model, T, precision)
    if t:
        ctx.set_tuning(**t)
    return t


def server_table(table: dict | None = None):
    """[(model, lg, precision, schedule)] for every tuned class."""
    tab = table if table is not None else load_cache()
    return [(r["model"], r["lg"], r["precision"], r["best"]) for r in tab.get("classes", {}).values()]


def time_schedule(ctx, opts, precision, reps=4):
    """Median wall time of `reps` launches after one warmup (launch times vary by several per cent with the
    order in which workgroups meet the work pool, so a single best launch ranks schedules poorly)."""
    import torch

    from paper_2303_02317_amd import binding

    ws = torch.empty(binding.workspace_bytes(opts, precision), dtype=torch.uint8, device="cuda")
    binding.launch_batch(ctx, opts, precision=precision, workspace=ws)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        L = binding.launch_batch(ctx, opts, precision=precision, workspace=ws)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return sorted(times)[len(times) // 2], L.price.cpu().numpy()


def tune(ctx, classes=DEFAULT_CLASSES, precision=0, n_options=64, candidates=CANDIDATES, log=print) -> dict:
    import numpy as np

    from paper_2303_02317_amd import inputs

    base = ctx.tuning()
    table = {"arch": "gfx950", "generated_by": "paper_2303_02317_amd.autotune", "n_options": n_options,
             "classes": {}}
    for model, lg in classes:
        opts = inputs.batch(CONFIG_ID[model], lg, n_options, model)
        rows, ref = [], None
        for cand in candidates:
            cand = dict(SCHEDULE_DEFAULTS, **cand)
            ctx.set_tuning(**dict(base, **cand))
            sec, prices = time_schedule(ctx, opts, precision)
            if ref is None:
                ref = prices
            K = np.array([o["K"] for o in opts])
            err = np.abs(prices - ref)
            rel = np.where(np.abs(ref) >= 1e-3 * K, err / np.maximum(np.abs(ref), 1e-300), 0.0)
            small = np.where(np.abs(ref) < 1e-3 * K, err / K, 0.0)
            same = bool(np.all(np.isfinite(prices)) and rel.max() <= 1e-9 and small.max() <= 1e-13)
            rows.append(dict(cand, seconds=sec, same_prices=same, max_rel_vs_first=float(rel.max())))
            log("class m%d lg%d p%d %s: %.2f ms, max rel diff %.1e%s" % (model, lg, precision, cand, sec * 1e3,
                                                                     rel.max(), "" if same else " REJECTED"))
        ok = [r for r in rows if r["same_prices"]]
        best = min(ok, key=lambda r: r["seconds"])
        if rows[0]["same_prices"] and best["seconds"] > (1.0 - NOISE) * rows[0]["seconds"]:
            best = rows[0]  # within launch-to-launch noise of the default: keep the default
        table["classes"][class_key(model, lg, precision)] = {
            "model": model, "lg": lg, "precision": precision,
            "best": {k: best[k] for k in SCHEDULE_KEYS},
            "noise_threshold": NOISE,
            "timings_ms": [dict({k: r[k] for k in SCHEDULE_KEYS}, ms=1e3 * r["seconds"],
                                max_rel_vs_first=r["max_rel_vs_first"]) for r in rows],
        }
    ctx.set_tuning(**base)
    return table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=CACHE)
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--options", type=int, default=64)
    ap.add_argument("--classes", default="", help="comma list of model:log2T, default the benchmark workloads")
    args = ap.parse_args()
    from paper_2303_02317_amd import binding

    classes = DEFAULT_CLASSES
    if args.classes:
        classes = [tuple(int(v) for v in c.split(":")) for c in args.classes.split(",")]
    ctx = binding.Context(0)
    table = tune(ctx, classes, args.precision, args.options)
    old = load_cache(args.out)
    old.setdefault("classes", {}).update(table["classes"])
    for k in ("arch", "generated_by", "n_options"):
        old[k] = table[k]
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(old, f, indent=1, sort_keys=True)
    print("wrote", args.out)
    ctx.close()


if __name__ == "__main__":
    main()
