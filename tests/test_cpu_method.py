"""The host multicore form of the method (libaop_cpu: OpenMP tasks, the
paper's own setting) against the CPU oracle: prices within the FP64 parity
tolerance, boundaries equal except at the oracle's near-ties, results
independent of the thread count and of the base-case size beyond rounding."""
import numpy as np
import pytest

from paper_2303_02317_amd import inputs
from tests import parity

B, TR, P = 0, 1, 2


@pytest.fixture(scope="module")
def cpu():
    from paper_2303_02317_amd import build, cpu as cpu_mod

    if not __import__("os").path.exists(cpu_mod.LIB_PATH):
        build.build_cpu()
    return cpu_mod


def _check(oracle_mod, opts, p, st, b):
    refs = oracle_mod.price_many(opts, boundary=True, margin=True)
    fails = []
    for k, (o, (ref, ob, mg)) in enumerate(zip(opts, refs)):
        assert st[k] == 0, (o, st[k])
        if not parity.price_ok(p[k], ref, o["K"]):
            fails.append(("price", o, p[k], ref))
        bad = parity.boundary_mismatches(b[k][:o["T"] + 1], ob, mg, o["model"], o["T"])
        if bad:
            fails.append(("boundary", o, bad[:4]))
    assert not fails, fails[:4]


@pytest.mark.parametrize("model", [B, TR, P])
def test_cpu_method_matches_oracle(cpu, oracle_mod, model):
    opts = []
    for T in (1, 2, 3, 5, 31, 64, 65, 100, 257, 1000, 2047, 4100):
        opts += inputs.batch(900 + model, T % 64, 3, model, T=T)
    p, st, b = cpu.price_batch(opts, threads=4, boundary=True)
    _check(oracle_mod, opts, p, st, b)


EDGE = [
    (100.0, 100.0, 0.05, 0.03, 0.2, 1.0),    # the single-option point (tie at expiry)
    (150.0, 50.0, 0.01, 0.06, 0.1, 2.0),     # immediate exercise
    (50.0, 150.0, 0.08, 0.01, 0.5, 0.25),    # tiny price
    (140.0, 60.0, 0.08, 0.0, 0.3, 1.0),      # Y = 0: one tilted correlation
    (100.0, 100.0, 0.05, 1e-4, 0.2, 1.0),    # nearly all continuation
]


@pytest.mark.parametrize("model", [B, TR, P])
@pytest.mark.parametrize("base", [2, 8, 64])
def test_cpu_method_edges_and_base_sizes(cpu, oracle_mod, model, base):
    opts = [inputs.option(model, S, K, r, 0.0 if model == P else q, s, E, T)
            for (S, K, r, q, s, E) in EDGE for T in (63, 130, 1001, 3000)]
    p, st, b = cpu.price_batch(opts, threads=2, base=base, boundary=True)
    _check(oracle_mod, opts, p, st, b)


def test_cpu_method_thread_count_does_not_change_results(cpu):
    opts = []
    for m in (B, TR, P):
        opts += inputs.batch(910 + m, 15, 3, m, T=20000 + 5000 * m)
    p1, _, b1 = cpu.price_batch(opts, threads=1, boundary=True)
    p4, _, b4 = cpu.price_batch(opts, threads=4, boundary=True)
    assert np.array_equal(p1, p4) and np.array_equal(b1, b4)


def test_cpu_method_european_and_rejections(cpu, oracle_mod):
    opts = [dict(o, european=True) for m in (B, TR, P) for o in inputs.batch(920 + m, 9, 3, m, T=1500)]
    p, st, _ = cpu.price_batch(opts)
    for k, o in enumerate(opts):
        assert st[k] == 0 and parity.price_ok(p[k], oracle_mod.price_option(o, american=False), o["K"])
    bad = [dict(inputs.CONFIG1, S0=-1.0), dict(inputs.CONFIG1, model=2), dict(inputs.CONFIG1, model=1, r=-0.01, q=0.0)]
    p, st, _ = cpu.price_batch(bad)
    assert list(st) == [1, 1, 2] and np.isnan(p).all()


def test_cpu_method_single_option_point(cpu, oracle_mod):
    p, _, b = cpu.price_batch([dict(inputs.CONFIG1)], boundary=True)
    assert p[0] == pytest.approx(8.65179401413394, rel=1e-12)
    assert b[0][2000] == 1000 and b[0][1999] == 1056
