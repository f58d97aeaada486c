"""The entry point that allocates nothing (aop_price_batch_noalloc) against
aop_price_batch on the same options: identical prices, statuses and
boundaries on two calls in a row, the second with a smaller batch, and
refusal (before any launch) of requests beyond the fixed scratch."""
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


def both(ctx, opts, precision=0):
    import torch

    from paper_2303_02317_amd import binding

    assert binding.workspace_bytes(opts, precision) <= binding.load().aop_noalloc_scratch_bytes()
    say("noalloc batch:", len(opts), "options, T up to", max(o["T"] for o in opts), "precision", precision)
    pn, sn, bn = binding.launch_batch_noalloc(ctx, opts, precision=precision, boundary=True)
    torch.cuda.synchronize()
    pn, bn = pn.cpu().numpy(), bn.cpu().numpy()
    say("reference batch through aop_price_batch")
    pr, sr, br = binding.price_batch(ctx, opts, precision=precision, boundary=True)
    return (pn, sn, bn), (pr, sr, br)


def check_same(opts, got, ref):
    pn, sn, bn = got
    pr, sr, br = ref
    assert list(sn) == list(sr)
    for k, o in enumerate(opts):
        if sr[k] != 0:
            assert np.isnan(pn[k]) and np.isnan(pr[k])
            continue
        assert pn[k] == pr[k], (o, pn[k], pr[k])  # same kernels, same schedule: bitwise
        T = o["T"]
        assert np.array_equal(bn[k][:T + 1], br[k][:T + 1]), o


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_price_batch_twice(ctx, precision):
    big = []
    for m in (0, 1, 2):
        big += inputs.batch(790 + m, 13, 5, m, T=9000 + 3000 * m)
    big.append(dict(inputs.CONFIG1, sigma=-1.0))  # rejected on the host: status, NaN
    small = inputs.batch(795, 9, 3, 0, T=700) + inputs.batch(796, 9, 2, 2, T=500)
    for opts in (big, small):  # the second call is smaller and reuses the scratch
        got, ref = both(ctx, opts, precision)
        check_same(opts, got, ref)


def test_noalloc_refuses_beyond_scratch(ctx):
    from paper_2303_02317_amd import binding

    cap = binding.load().aop_noalloc_scratch_bytes()
    huge = inputs.batch(797, 20, 1, 1)  # one trinomial option of T = 2^20: more than the scratch
    assert binding.workspace_bytes(huge) > cap
    with pytest.raises(binding.AopError, match="memory"):
        binding.launch_batch_noalloc(ctx, huge)
    many = inputs.batch(798, 5, 257, 0, T=32)  # more options than the entry point stages
    with pytest.raises(binding.AopError, match="memory"):
        binding.launch_batch_noalloc(ctx, many)
    # still usable afterwards
    opts = inputs.batch(799, 8, 4, 0, T=300)
    got, ref = both(ctx, opts)
    check_same(opts, got, ref)
