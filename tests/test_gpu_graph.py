"""GPU test of the hipGraph form of a batch launch (aop_graph_*).

The graph is replayed several times with eager work and synchronisations in
between; every replay must reproduce the eager prices bitwise, and those
prices must match the CPU oracle.
"""
import numpy as np
import pytest

from paper_2303_02317_amd import inputs
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_02317_amd import binding

    c = binding.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replays_match_eager(ctx, oracle_mod, precision):
    import torch

    from paper_2303_02317_amd import binding

    opts = []
    for m in (0, 1, 2):
        opts += inputs.batch(780 + m, 13, 4, m, T=3000 + 2000 * m)
    ref, st, rb = binding.price_batch(ctx, opts, precision=precision, boundary=True)
    assert (st == 0).all()
    rel, ak = (parity.REL_FP64, parity.ABS_FP64_K) if precision == 0 else (parity.REL_MIXED, parity.ABS_MIXED_K)
    for i, (o, (orc, ob, mg)) in enumerate(zip(opts, oracle_mod.price_many(opts, boundary=True, margin=True))):
        assert parity.price_ok(ref[i], orc, o["K"], rel, ak), (o, ref[i], orc)
        assert not parity.boundary_mismatches(rb[i][:o["T"] + 1], ob, mg, o["model"], o["T"])
    g = binding.BatchGraph(ctx, opts, precision=precision, boundary=True)
    other = inputs.batch(790, 11, 5, 1)
    for k in range(8):
        g.price.fill_(float("nan"))
        g.boundary.fill_(-7)
        p = g.launch()
        torch.cuda.synchronize()
        got = p.cpu().numpy()
        if not np.array_equal(got, ref):
            print("replay", k, "errors", binding.batch_errors(g, g.n), "pool", binding.pool_stats(g, g.n),
                  "stats", binding.batch_stats(g, g.n)[:, :4], flush=True)
        assert np.array_equal(got, ref), (k, got, ref)
        for i, o in enumerate(opts):
            assert np.array_equal(g.boundary[i].cpu().numpy()[:o["T"] + 1], rb[i][:o["T"] + 1])
        # eager work between replays
        binding.price_batch(ctx, other)
        torch.cuda.synchronize()
    g.close()
