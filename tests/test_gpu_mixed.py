"""GPU parity of the mixed-precision path (split FP32 correlations, FP64 band,
boundary and root) with the FP64 CPU oracle.

The tolerance is the mixed one of ``tests/parity.py`` (1e-6 relative, or 1e-9 K
absolute for prices below 1e-3 K); every option's absolute and relative
error is printed.  Boundaries are checked with the same near-tie rule as the
FP64 path: the band and the boundary decisions run in FP64 either way.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_2303_02317_amd import inputs
from tests import parity

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_02317_amd import binding

    c = binding.Context(0)
    yield c
    c.close()


def mixed_ok(got, ref, K):
    return parity.price_ok(got, ref, K, parity.REL_MIXED, parity.ABS_MIXED_K)


def run_mixed(ctx, opts, boundary=True):
    from paper_2303_02317_amd import binding

    say("gpu mixed batch:", len(opts), "options, models", sorted({o["model"] for o in opts}),
        "T in", sorted({o["T"] for o in opts})[:6])
    return binding.price_batch(ctx, opts, precision=binding.AOP_MIXED, boundary=boundary)


@pytest.mark.parametrize("model", [0, 1, 2])
def test_mixed_small_T(ctx, oracle_mod, model):
    opts = []
    for T in (5, 64, 65, 300, 1000, 2049, 4100, 9000):
        opts += inputs.batch(740 + model, T % 64, 3, model, T=T)
    p, s, b = run_mixed(ctx, opts)
    refs = oracle_mod.price_many(opts, boundary=True, margin=True)
    fails = []
    for k, (o, (ref, ob, mg)) in enumerate(zip(opts, refs)):
        assert s[k] == 0
        ae, re = parity.price_errors(p[k], ref)
        say("model %d T %5d price %.12g abs/K %.2e rel %.2e" % (model, o["T"], ref, ae / o["K"], re))
        if not mixed_ok(p[k], ref, o["K"]):
            fails.append(("price", o, p[k], ref, ae, re))
        bad = parity.boundary_mismatches(b[k][:o["T"] + 1], ob, mg, o["model"], o["T"])
        if bad:
            fails.append(("boundary", o, bad[:5], len(bad)))
    assert not fails, fails[:4]


def test_mixed_close_to_fp64_path(ctx):
    # Same options through both paths: the mixed prices stay within the mixed
    # tolerance of the FP64 ones.
    from paper_2303_02317_amd import binding

    opts = []
    for m in (0, 1, 2):
        opts += inputs.batch(750 + m, 12, 4, m)
    p64, _, _ = binding.price_batch(ctx, opts, precision=binding.AOP_FP64)
    pmx, _, _ = run_mixed(ctx, opts, boundary=False)
    for k, o in enumerate(opts):
        assert mixed_ok(pmx[k], p64[k], o["K"]), (o, pmx[k], p64[k])


GOLDEN = ["oracle_trinomial_c3_t16.json", "oracle_bsm_c4_t16.json", "oracle_binomial_c2_t17.json",
          "oracle_trinomial_c3_t18.json", "oracle_bsm_c4_t18.json", "oracle_trinomial_c3_t20.json"]


@pytest.mark.parametrize("fname", GOLDEN)
def test_mixed_golden(ctx, fname):
    path = os.path.join(HERE, "golden", fname)
    doc = json.load(open(path))
    recs = doc["options"]
    opts = [r["params"] for r in recs]
    p, st, b = run_mixed(ctx, opts, boundary=True)
    fails, rels = [], []
    for k, r in enumerate(recs):
        o = r["params"]
        assert st[k] == 0, (k, st[k])
        ae, re = parity.price_errors(p[k], r["price"])
        say("%s option %d: price %.12g abs/K %.2e rel %.2e" % (fname, k, r["price"], ae / o["K"], re))
        mg = parity.golden_margins(r)
        if mg is not None:
            rows = np.asarray(r["boundary_rows"])
            bad = parity.boundary_mismatches(b[k][rows], np.asarray(r["boundary"], dtype=np.int64), mg,
                                             o["model"], o["T"])
            if bad:
                fails.append(("boundary", k, bad[:5]))
        if abs(r["price"]) >= 1e-3 * o["K"]:
            rels.append(re)
        if not mixed_ok(p[k], r["price"], o["K"]):
            fails.append((k, p[k], r["price"], ae, re))
    say(fname, "mixed: max rel err (price >= 1e-3 K) %.3e over %d options" % (max(rels), len(rels)))
    assert not fails, fails[:4]
