"""Failure handling on the GPU: a launch whose waits pass their deadline.

The host sets a 2 microsecond deadline (``aop_tuning.timeout_us``) on a batch
of binomial options of T = 2^20: one FFT tile alone takes several
microseconds, so a driver that waits for a helper's tile passes it.  Every wait
of the launch is bounded by that deadline, so the launch ends on its own (the
waits return once the pool's abort flag is set, and the helpers leave): an option whose wait
expired prices NaN with its device error (timeout or abort), the pool records
the first cause, and an option that finished before the abort carries the
stored oracle price.  The same context then prices the batch correctly with
the normal deadline (the pool is cleared at each launch).
"""
import json
import math
import os
import sys

import numpy as np
import pytest

from tests import parity

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
DEV_TIMEOUT, DEV_ABORT = 5, 6


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


def test_expired_deadline_aborts_cleanly_then_recovers(ctx):
    import torch

    from paper_2303_02317_amd import binding

    doc = json.load(open(os.path.join(HERE, "golden", "oracle_binomial_c2_t20.json")))
    recs = doc["options"][:4]
    opts = [dict(r["params"]) for r in recs]
    ref = [r["price"] for r in recs]
    try:
        ctx.set_tuning(timeout_us=2)
        say("deadline 2 us: binomial T=2^20,", len(opts), "options")
        L = binding.launch_batch(ctx, opts)
        torch.cuda.synchronize()
        p = L.price.cpu().numpy()
        errs = binding.batch_errors(L, len(opts))
        info = binding.pool_abort_info(L, len(opts))
        say("prices", p.tolist(), "errors", errs.tolist(), "abort", info)
    finally:
        ctx.set_tuning(timeout_us=0)
    assert list(L.status) == [0] * len(opts)  # accepted on the host; failures are per option on the device
    for k in range(len(opts)):
        if math.isnan(p[k]):
            assert errs[k] in (DEV_TIMEOUT, DEV_ABORT), (k, errs[k])
        else:
            assert errs[k] == 0 and parity.price_ok(p[k], ref[k], opts[k]["K"]), (k, p[k], ref[k])
    if not np.isnan(p).any():
        pytest.skip("every wait finished within the deadline: nothing to abort")
    # a wait on the pool (2) or a drain (3) that expired aborts the whole
    # launch and is recorded; a wave-level wait that expired fails its own
    # option only (DEV_TIMEOUT), without a pool abort
    reason = list(info.values())[0]
    assert reason in (0, 2, 3), info
    if reason == 0:
        assert all(e != DEV_ABORT for e in errs.tolist()), (errs, info)

    say("normal deadline: the same batch")
    L = binding.launch_batch(ctx, opts)
    torch.cuda.synchronize()
    p = L.price.cpu().numpy()
    errs = binding.batch_errors(L, len(opts))
    assert errs.tolist() == [0] * len(opts)
    for k in range(len(opts)):
        assert parity.price_ok(p[k], ref[k], opts[k]["K"]), (k, p[k], ref[k])
