"""Write oracle prices for the large seeded workloads (calls only ``oracle/``).

The plain Theta(T^2) oracle needs minutes per option at T = 2^20, far too long
for a test run, so its results for the benchmark workloads are stored here:

    oracle_<model>_c<config>_t<log2T>.json

Each file holds, per option, the parameters, the American price and the
oracle's boundary at a fixed set of sampled rows.  Inputs come from
``paper_2303_02317_amd.inputs.batch(config, log2T, 64, model)``; a file may hold
only the first k options of the 64 (stated in the file as ``n_options``).

Usage: python tests/golden/make_golden.py [--threads N] [--only name ...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2303_02317_amd import inputs  # noqa: E402

# (name, model, config id, log2T, number of options)
JOBS = [
    ("binomial", 0, 2, 14, 64),
    ("trinomial", 1, 3, 16, 64),
    ("bsm", 2, 4, 16, 64),
    ("binomial", 0, 2, 17, 64),
    ("trinomial", 1, 3, 18, 24),
    ("bsm", 2, 4, 18, 24),
    ("binomial", 0, 2, 20, 12),
    ("trinomial", 1, 3, 20, 6),
]


def sample_rows(T: int) -> list[int]:
    rows = {0, 1, 2, T - 2, T - 1, T}
    for k in range(1, 25):
        rows.add(int(round(T * k / 25.0)))
    return sorted(r for r in rows if 0 <= r <= T)


def run_one(opt):
    t0 = time.time()
    price, b, _ = oracle.price_option(opt, boundary=True)
    dt = time.time() - t0
    rows = sample_rows(opt["T"])
    return dict(params=opt, price=price, seconds=dt,
                boundary_rows=rows, boundary=[int(b[r]) for r in rows])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=len(os.sched_getaffinity(0)))
    ap.add_argument("--only", nargs="*", default=None)
    args = ap.parse_args()
    oracle.build()
    for name, model, cfg, log2T, n in JOBS:
        fname = "oracle_%s_c%d_t%d.json" % (name, cfg, log2T)
        if args.only and fname not in args.only and name not in args.only:
            continue
        path = os.path.join(HERE, fname)
        if os.path.exists(path):
            continue
        opts = inputs.batch(cfg, log2T, 64, model)[:n]
        t0 = time.time()
        with ThreadPoolExecutor(max_workers=args.threads) as ex:
            recs = list(ex.map(run_one, opts))
        doc = dict(model=model, config=cfg, log2T=log2T, T=1 << log2T, n_options=n,
                   seed=[cfg, log2T], lam=oracle.DEFAULT_LAMBDA, threads=args.threads,
                   wall_seconds=time.time() - t0, options=recs)
        with open(path + ".tmp", "w") as f:
            json.dump(doc, f, indent=1)
        os.replace(path + ".tmp", path)
        print("wrote", fname, "in %.1fs" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
