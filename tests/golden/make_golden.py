"""Write oracle prices for the large seeded workloads (calls only ``oracle/``).

The plain Theta(T^2) oracle needs minutes per option at T = 2^20, far too long
for a test run, so its results for the benchmark workloads are stored here:

    oracle_<model>_c<config>_t<log2T>.json

Each file holds, per option, the parameters, the American price, and at a
fixed set of sampled rows the oracle's boundary together with its decision
margins there (the gap at the boundary cell and at the cell after it, in the
oracle's units: K for the lattices, the nondimensional value for BSM; null
where the oracle reports none).  Inputs come from
``paper_2303_02317_amd.inputs.batch(config, log2T, 64, model)``; a file may
hold only the first k options of the 64 (stated in the file as
``n_options``).

Options are priced in parallel, one per thread; each finished option is
cached under ``--cache`` so that an interrupted run resumes where it stopped.
``--partial`` prices nothing: it writes each file with the longest run of
options 0, 1, ... found in the cache, where that extends the stored file.

Usage: python tests/golden/make_golden.py [--threads N] [--only name ...]
                                          [--cache DIR] [--partial]
       python tests/golden/make_golden.py --european   (European lattice sums)
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import threading
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2303_02317_amd import inputs  # noqa: E402

# (name, model, config id, log2T, number of options)
JOBS = [
    ("binomial", 0, 2, 14, 64),
    ("trinomial", 1, 3, 16, 64),
    ("bsm", 2, 4, 16, 64),
    ("binomial", 0, 2, 17, 64),
    ("bsm", 2, 4, 18, 64),
    ("trinomial", 1, 3, 18, 64),
    ("binomial", 0, 2, 20, 64),
    ("trinomial", 1, 3, 20, 24),
]


def sample_rows(T: int) -> list[int]:
    rows = {0, 1, 2, T - 2, T - 1, T}
    for k in range(1, 25):
        rows.add(int(round(T * k / 25.0)))
    return sorted(r for r in rows if 0 <= r <= T)


def _num(x: float):
    return float(x) if math.isfinite(x) else (None if math.isnan(x) else ("-inf" if x < 0 else "inf"))


def run_one(opt):
    t0 = time.time()
    price, b, mg = oracle.price_option(opt, boundary=True, margin=True)
    dt = time.time() - t0
    rows = sample_rows(opt["T"])
    return dict(params=opt, price=price, seconds=dt, boundary_rows=rows,
                boundary=[int(b[r]) for r in rows],
                margin=[[_num(mg[2 * r]), _num(mg[2 * r + 1])] for r in rows])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=len(os.sched_getaffinity(0)))
    ap.add_argument("--only", nargs="*", default=None)
    ap.add_argument("--cache", default=os.path.join(HERE, "cache"))
    ap.add_argument("--partial", action="store_true")
    args = ap.parse_args()
    oracle.build()
    os.makedirs(args.cache, exist_ok=True)
    lock = threading.Lock()
    for name, model, cfg, log2T, n in JOBS:
        fname = "oracle_%s_c%d_t%d.json" % (name, cfg, log2T)
        if args.only and fname not in args.only and name not in args.only:
            continue
        path = os.path.join(HERE, fname)
        if os.path.exists(path):
            doc = json.load(open(path))
            if doc.get("n_options", 0) >= n and all("margin" in r for r in doc["options"]):
                continue
        cache = os.path.join(args.cache, fname + ".jsonl")
        done = {}
        if os.path.exists(cache):
            for line in open(cache):
                rec = json.loads(line)
                done[rec["index"]] = rec["record"]
        opts = inputs.batch(cfg, log2T, 64, model)[:n]
        if args.partial:
            k = 0
            while k < n and k in done:
                k += 1
            have = json.load(open(path)).get("n_options", 0) if os.path.exists(path) else 0
            if k > have:
                assert all(done[i]["params"] == opts[i] for i in range(k))
                doc = dict(model=model, config=cfg, log2T=log2T, T=1 << log2T, n_options=k,
                           seed=[cfg, log2T], lam=oracle.DEFAULT_LAMBDA, threads=args.threads,
                           wall_seconds=sum(done[i]["seconds"] for i in range(k)),
                           options=[done[i] for i in range(k)])
                with open(path + ".tmp", "w") as f:
                    json.dump(doc, f, indent=1)
                os.replace(path + ".tmp", path)
                print("wrote", fname, "with the first", k, "options", flush=True)
            continue
        todo = [k for k in range(n) if k not in done]
        t0 = time.time()

        def work(k):
            rec = run_one(opts[k])
            with lock:
                with open(cache, "a") as f:
                    f.write(json.dumps(dict(index=k, record=rec)) + "\n")
                print("%s option %d: %.1fs" % (fname, k, rec["seconds"]), flush=True)
            return k, rec

        with ThreadPoolExecutor(max_workers=args.threads) as ex:
            for k, rec in ex.map(work, todo):
                done[k] = rec
        doc = dict(model=model, config=cfg, log2T=log2T, T=1 << log2T, n_options=n,
                   seed=[cfg, log2T], lam=oracle.DEFAULT_LAMBDA, threads=args.threads,
                   wall_seconds=time.time() - t0, options=[done[k] for k in range(n)])
        with open(path + ".tmp", "w") as f:
            json.dump(doc, f, indent=1)
        os.replace(path + ".tmp", path)
        print("wrote", fname, "in %.1fs" % (time.time() - t0), flush=True)


# European calls on the lattices at full size: the oracle's O(T) closed-form
# sums (oracle.european_sum), pinned against its plain induction.
EUROPEAN_JOBS = [
    ("binomial", 0, 2, 20, 64),
    ("trinomial", 1, 3, 20, 64),
]


def write_european():
    for name, model, cfg, log2T, n in EUROPEAN_JOBS:
        fname = "oracle_european_%s_c%d_t%d.json" % (name, cfg, log2T)
        path = os.path.join(HERE, fname)
        if os.path.exists(path) and json.load(open(path)).get("n_options", 0) >= n:
            continue
        opts = inputs.batch(cfg, log2T, 64, model)[:n]
        t0 = time.time()
        recs = []
        for o in opts:
            price = oracle.european_sum(model, o["S0"], o["K"], o["r"], o["q"], o["sigma"], o["expiry"], o["T"])
            recs.append(dict(params=dict(o, european=True), price=price))
        doc = dict(model=model, config=cfg, log2T=log2T, T=1 << log2T, n_options=n, seed=[cfg, log2T],
                   european=True, method="closed-form sum over the up-move distribution",
                   wall_seconds=time.time() - t0, options=recs)
        with open(path + ".tmp", "w") as f:
            json.dump(doc, f, indent=1)
        os.replace(path + ".tmp", path)
        print("wrote", fname, "in %.1fs" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--european":
        oracle.build()
        write_european()
    else:
        main()
