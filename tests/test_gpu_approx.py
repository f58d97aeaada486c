"""GPU parity of the Gaussian approximations of the European binomial call
(the paper's section on the European call under the binomial model) with the
oracle's evaluation of the same formulas, plus their error against the exact
European lattice value (reported, with the 1/T convergence the oracle pins)."""
import sys

import numpy as np
import pytest

from paper_2303_02317_amd import inputs

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("method", [0, 1, 2])
def test_approx_matches_oracle_formulas(ctx, oracle_mod, method):
    from paper_2303_02317_amd import binding

    opts = []
    for T in (1, 2, 7, 64, 1000, 4097, 1 << 16, 1 << 20):
        opts += inputs.batch(830, T % 64, 4, 0, T=T)
    opts.append(inputs.option(0, 150.0, 50.0, 0.01, 0.06, 0.1, 2.0, 5000))  # deep in the money
    opts.append(inputs.option(0, 50.0, 150.0, 0.08, 0.01, 0.5, 0.25, 5000))  # deep out of the money
    say("approx method", method, len(opts), "options")
    p, st = binding.european_approx(ctx, opts, method)
    fails = []
    for k, o in enumerate(opts):
        assert st[k] == 0
        ref = oracle_mod.european_gauss(method, o["S0"], o["K"], o["r"], o["q"], o["sigma"], o["expiry"], o["T"])
        # same formula, summed in another order (sums) or with the device erf
        if not abs(p[k] - ref) <= 1e-11 * max(abs(ref), 1e-3 * o["K"]):
            fails.append((o, p[k], ref))
    assert not fails, fails[:4]


def test_approx_error_against_exact_lattice(ctx, oracle_mod):
    # Error study at T = 2^20 on the binomial workload: every method within
    # the accuracy the oracle pins for it (1/T-order sums, coarser erf form).
    from paper_2303_02317_amd import binding

    opts = inputs.batch(2, 20, 16, 0)
    exact = np.array([oracle_mod.european_sum(0, o["S0"], o["K"], o["r"], o["q"], o["sigma"], o["expiry"], o["T"])
                      for o in opts])
    big = exact >= 1e-3 * np.array([o["K"] for o in opts])
    for method, bound in ((0, 1e-5), (1, 1e-5), (2, 1e-3)):
        p, st = binding.european_approx(ctx, opts, method)
        assert (st == 0).all()
        rel = np.abs(p - exact)[big] / exact[big]
        say("method", method, "max rel err vs exact lattice", rel.max())
        assert rel.max() <= bound


def test_approx_rejects_other_models(ctx):
    from paper_2303_02317_amd import binding

    opts = [inputs.option(1, 100, 100, 0.05, 0.02, 0.2, 1.0, 100), inputs.option(0, 100, 100, 0.05, 0.02, 0.2, 1.0, 100),
            inputs.option(0, -1, 100, 0.05, 0.02, 0.2, 1.0, 100)]
    p, st = binding.european_approx(ctx, opts, 1)
    assert list(st) == [7, 0, 1] and np.isnan(p[0]) and np.isfinite(p[1]) and np.isnan(p[2])
