"""GPU tests of the continuous-batching server (aop_server_*).

Requests of mixed model and T arrive while earlier batches are on the device;
every result must be bitwise the price the same option gets alone (each
option's schedule depends only on that option), and match the oracle.
"""
import sys
import time

import numpy as np
import pytest

from paper_2303_02317_amd import inputs
from tests import parity

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


def torch_sync():
    import torch

    torch.cuda.synchronize()


def drain(srv, n, timeout_s=60.0):
    got = {}
    t0 = time.time()
    while len(got) < n:
        for r in srv.poll(4096, 2000):
            got[r["id"]] = r
        assert time.time() - t0 < timeout_s, ("server stalled", len(got), n, srv.stats())
    return got


def serve_stream(srv, opts, rate_per_s, seed):
    # Poisson arrivals: submit each request at its arrival time while results come back
    arr = inputs.poisson_arrivals(len(opts), rate_per_s, seed=seed)
    t0 = time.perf_counter()
    got = {}
    k = 0
    while k < len(opts):
        now = time.perf_counter() - t0
        j = k
        while j < len(opts) and arr[j] <= now:
            j += 1
        if j > k:
            srv.submit(opts[k:j], list(range(k, j)))
            k = j
        for r in srv.poll(4096, 0):
            got[r["id"]] = r
        time.sleep(0.0005)
    got.update(drain(srv, len(opts) - len(got)) if len(got) < len(opts) else {})
    return got


@pytest.mark.parametrize("precision", [0, 1])
def test_serve_mix_equals_alone(ctx, oracle_mod, precision):
    from paper_2303_02317_amd import binding

    opts = inputs.serving_mix(36, seed=(760 + precision, 0), log2T_lo=8.0, log2T_hi=13.0)
    srv = binding.Server(ctx, hbm_budget=1 << 30, max_inflight=3, max_batch=6, precision=precision)
    say("serve: %d requests, precision %d" % (len(opts), precision))
    got = serve_stream(srv, opts, rate_per_s=400.0, seed=(761, precision))
    st = srv.stats()
    srv.close()
    say("server stats", st)
    assert st["completed"] == len(opts) and st["batches"] >= 2
    L = binding.launch_batch(ctx, opts, precision=precision)  # same schedule per option
    torch_sync()
    alone = L.price.cpu().numpy()
    errs = binding.batch_errors(L, len(opts))
    if (errs != 0).any() or not np.isfinite(alone).all():
        say("batch of the whole mix: errors", errs.tolist(), "pool", binding.pool_stats(L, len(opts)), "abort", binding.pool_abort_info(L, len(opts)))
    assert (errs == 0).all(), errs
    refs = oracle_mod.price_many(opts)
    tol = (parity.REL_MIXED, parity.ABS_MIXED_K) if precision else (parity.REL_FP64, parity.ABS_FP64_K)
    lat = []
    for i, o in enumerate(opts):
        r = got[i]
        assert r["status"] == 0, r
        single = binding.price_batch(ctx, [o], precision=precision)[0][0]
        assert r["price"] == single, (i, o, r["price"], single)
        assert r["price"] == alone[i]
        assert parity.price_ok(r["price"], refs[i], o["K"], *tol), (o, r["price"], refs[i])
        assert 0.0 <= r["queue_s"] <= r["latency_s"]
        lat.append(r["latency_s"])
    say("latency p50 %.2f ms p99 %.2f ms" % (1e3 * np.percentile(lat, 50), 1e3 * np.percentile(lat, 99)))


def test_serve_admission_by_budget(ctx):
    from paper_2303_02317_amd import binding

    opts = inputs.batch(770, 12, 12, 0)  # 12 binomial options at T = 4096
    two = binding.workspace_bytes(opts[:2])  # a two-option batch (work pool included)
    area = two - binding.workspace_bytes(opts[:1])  # one more option's own area
    budget = two + area // 2  # room for one two-option batch at a time
    srv = binding.Server(ctx, hbm_budget=budget, max_inflight=4, max_batch=8)
    srv.submit(opts, list(range(len(opts))))
    got = drain(srv, len(opts))
    st = srv.stats()
    srv.close()
    say("admission stats", st, "budget", budget)
    assert st["peak_bytes"] <= st["arena_bytes"]
    assert st["batches"] >= 6  # the budget forces two-option batches
    alone, _, _ = binding.price_batch(ctx, opts)
    for i in range(len(opts)):
        assert got[i]["status"] == 0 and got[i]["price"] == alone[i]


def test_serve_refuses_invalid_and_oversized(ctx):
    from paper_2303_02317_amd import binding

    good = inputs.batch(771, 9, 2, 1, T=500)
    bad = dict(good[0], sigma=-0.1)
    huge = dict(good[0], T=1 << 20)
    srv = binding.Server(ctx, hbm_budget=64 << 20, max_inflight=2, max_batch=4)
    srv.submit([good[0], bad, huge, good[1]], [10, 11, 12, 13])
    got = drain(srv, 4)
    srv.close()
    assert got[11]["status"] == 1 and np.isnan(got[11]["price"])  # EINVAL at submission
    assert got[12]["status"] == 3 and np.isnan(got[12]["price"])  # larger than the whole budget
    alone, _, _ = binding.price_batch(ctx, [good[0], good[1]])
    assert got[10]["price"] == alone[0] and got[13]["price"] == alone[1]
