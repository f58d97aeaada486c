"""GPU parity of the plain Theta(T^2) stencil (the comparison path) with the oracle."""
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


@pytest.mark.parametrize("model", [0, 1, 2])
def test_plain_matches_oracle(ctx, oracle_mod, model):
    import torch

    from paper_2303_02317_amd import binding

    opts = []
    for T in (1, 2, 7, 63, 64, 65, 129, 1000, 1023, 1025, 3000):
        opts += inputs.batch(740 + model, T % 32, 2, model, T=T)
    print("plain batch model", model, len(opts), flush=True)
    L = binding.launch_plain(ctx, opts, boundary=True)
    torch.cuda.synchronize()
    p = L.price.cpu().numpy()
    b = L.boundary.cpu().numpy()
    refs = oracle_mod.price_many(opts, boundary=True, margin=True)
    for k, (o, (ref, ob, mg)) in enumerate(zip(opts, refs)):
        assert L.status[k] == 0
        # same arithmetic as the oracle up to FMA contraction and the
        # incrementally carried exercise values: far inside the FFT tolerance
        assert parity.price_ok(p[k], ref, o["K"], rel_tol=1e-12, abs_tol_k=1e-14), (o, p[k], ref)
        bad = parity.boundary_mismatches(b[k][:o["T"] + 1], ob, mg, model, o["T"])
        assert not bad, (o, bad[:5])


def test_plain_single_option_point_with_boundary(ctx, oracle_mod):
    # The single-option point (S = K = 100, R = 0.05, Y = 0.03, V = 0.2,
    # E = 1, T = 2000) on the plain GPU stencil: root and the boundary of
    # every row against the oracle (the expiry row has an exact tie at
    # column 1000, counted red).
    import torch

    from paper_2303_02317_amd import binding

    o = dict(inputs.CONFIG1)
    L = binding.launch_plain(ctx, [o], boundary=True)
    torch.cuda.synchronize()
    p, b = float(L.price.cpu().numpy()[0]), L.boundary.cpu().numpy()[0]
    ref, ob, mg = oracle_mod.price_option(o, boundary=True, margin=True)
    assert parity.price_ok(p, ref, o["K"], rel_tol=1e-12, abs_tol_k=1e-14), (p, ref)
    assert b[2000] == 1000 and b[1999] == 1056
    assert not parity.boundary_mismatches(b, ob, mg, 0, o["T"])


def test_plain_rejects_invalid(ctx):
    import torch

    from paper_2303_02317_amd import binding

    opts = [dict(inputs.CONFIG1), dict(inputs.CONFIG1, sigma=-1.0)]
    L = binding.launch_plain(ctx, opts)
    torch.cuda.synchronize()
    p = L.price.cpu().numpy()
    assert list(L.status) == [0, 1] and np.isfinite(p[0]) and np.isnan(p[1])
