"""GPU parity of the European pricer (one FFT correlation of the expiry row
with the multi-step stencil kernel; the paper's section on the European call
under the binomial model, for all three models) with the CPU oracle.

Small and medium T: the oracle's plain induction without exercise.  Full
size (T = 2^20, lattices): the oracle's O(T) sum over the up-move
distribution, pinned to that induction.  Boundary outputs: the expiry row's
entry as for the American option, -1 / INT64_MIN below it.
"""
import sys

import numpy as np
import pytest

from paper_2303_02317_amd import inputs
from tests import parity

pytestmark = pytest.mark.gpu
NONE = parity.BSM_NONE


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


def european(opts):
    return [dict(o, european=True) for o in opts]


def run(ctx, opts, precision=0, boundary=True):
    from paper_2303_02317_amd import binding

    say("gpu european batch:", len(opts), "options, models", sorted({o["model"] for o in opts}),
        "T in", sorted({o["T"] for o in opts})[:8], "precision", precision)
    return binding.price_batch(ctx, opts, precision=precision, boundary=boundary)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("model", [0, 1, 2])
def test_european_parity_small_T(ctx, oracle_mod, model, precision):
    opts = []
    for T in (1, 2, 5, 64, 65, 1000, 4100, 16384):
        opts += european(inputs.batch(760 + model, T % 64, 3, model, T=T))
    opts.append(dict(inputs.option(model, 140.0, 60.0, 0.08, 0.0, 0.3, 1.0, 3000), european=True))
    opts.append(dict(inputs.option(model, 100.0, 100.0, -0.01, 0.0, 0.3, 1.0, 2000), european=True))
    p, st, b = run(ctx, opts, precision)
    rel, ab = (parity.REL_FP64, parity.ABS_FP64_K) if precision == 0 else (parity.REL_MIXED, parity.ABS_MIXED_K)
    refs = oracle_mod.price_many(opts, american=False, boundary=True)
    fails = []
    for k, (o, (ref, ob, _)) in enumerate(zip(opts, refs)):
        assert st[k] == 0, (o, st[k])
        if not parity.price_ok(p[k], ref, o["K"], rel, ab):
            fails.append((o, p[k], ref, parity.price_errors(p[k], ref)))
        T = o["T"]
        # expiry row: the same split as the oracle's; below it no exercise boundary
        if model == 2:
            assert b[k][0] == ob[0] and all(b[k][1:T + 1] == NONE), o
        else:
            assert b[k][T] == ob[T] and all(b[k][:T] == -1), o
    assert not fails, fails[:4]


@pytest.mark.parametrize("model", [0, 1])
def test_european_full_size(ctx, oracle_mod, model):
    # T = 2^20, the seeded batches of the lattice workloads, against the
    # oracle's closed-form sums.
    opts = european(inputs.batch(2 if model == 0 else 3, 20, 16, model))
    p, st, _ = run(ctx, opts, boundary=False)
    worst = 0.0
    for k, o in enumerate(opts):
        ref = oracle_mod.european_sum(model, o["S0"], o["K"], o["r"], o["q"], o["sigma"], o["expiry"], o["T"])
        assert st[k] == 0
        assert parity.price_ok(p[k], ref, o["K"]), (o, p[k], ref)
        if abs(ref) >= 1e-3 * o["K"]:
            worst = max(worst, parity.price_errors(p[k], ref)[1])
    say("european T=2^20 model", model, "max rel err", worst)


@pytest.mark.parametrize("fname", ["oracle_european_binomial_c2_t20.json", "oracle_european_trinomial_c3_t20.json"])
def test_european_golden_full_size(ctx, fname):
    # All 64 options of each lattice workload at T = 2^20 against the stored
    # closed-form oracle sums (tests/golden/make_golden.py --european).
    import json
    import os

    doc = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", fname)))
    recs = doc["options"]
    opts = [r["params"] for r in recs]
    p, st, _ = run(ctx, opts, boundary=False)
    fails = [(k, p[k], r["price"]) for k, r in enumerate(recs)
             if st[k] != 0 or not parity.price_ok(p[k], r["price"], r["params"]["K"])]
    say(fname, "max rel err", max(parity.price_errors(p[k], r["price"])[1] for k, r in enumerate(recs)
                                  if abs(r["price"]) >= 1e-3 * r["params"]["K"]))
    assert not fails, fails[:4]


def test_european_and_american_in_one_batch(ctx):
    # Flags are per option: a mixed batch gives each option its solo price.
    from paper_2303_02317_amd import binding

    mix = []
    for m in (0, 1, 2):
        base = inputs.batch(770 + m, 11, 3, m, T=1500 + 500 * m)
        mix += base + european(base)
    pb, sb, _ = run(ctx, mix, boundary=False)
    assert (sb == 0).all()
    for k, o in enumerate(mix):
        pa, _, _ = binding.price_batch(ctx, [o])
        assert pa[0] == pb[k], (o, pa[0], pb[k])
    # the American price is never below the European one
    for k in range(0, len(mix), 6):
        for j in range(3):
            assert pb[k + j] >= pb[k + 3 + j] - 1e-12 * mix[k + j]["K"]


def test_plain_stencil_european(ctx, oracle_mod):
    from paper_2303_02317_amd import binding

    opts = []
    for m in (0, 1, 2):
        opts += european(inputs.batch(780 + m, 10, 3, m, T=700 + 400 * m))
    P = binding.launch_plain(ctx, opts)
    import torch

    torch.cuda.synchronize()
    pp = P.price.cpu().numpy()
    for k, o in enumerate(opts):
        ref = oracle_mod.price_option(o, american=False)
        assert abs(pp[k] - ref) <= 1e-12 * max(abs(ref), o["K"]), (o, pp[k], ref)
