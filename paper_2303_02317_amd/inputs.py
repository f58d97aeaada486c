"""Seeded synthetic option workloads.

This module only draws random option parameters; it holds none of the pricing
arithmetic.  Both the GPU path and the CPU oracle take their inputs from it.

Parameter ranges follow the synthetic experiments of arXiv 2303.02317
(Sec. 5 fixes S, K, R, V, Y, E and varies T; here they are drawn uniformly so
that every run covers in-, at- and out-of-the-money options, early-exercise
and immediate-exercise cases):

    S0, K ~ U[50, 150], r ~ U[0.01, 0.08], q ~ U[0.01, 0.06] (q = 0 for the
    BSM put, whose PDE carries no dividend), sigma ~ U[0.1, 0.5],
    expiry ~ U[0.25, 2] years.

A batch for (config id c, log2 T = t) uses ``numpy.random.default_rng([c, t])``
and draws per option, in this order: S0, K, r, q (not drawn for BSM), sigma,
expiry.
"""
from __future__ import annotations

import math

import numpy as np

BINOMIAL_CALL = 0
TRINOMIAL_CALL = 1
BSM_PUT = 2

#: Parameter set of the paper's experiments (Sec. 5, "Parameter Values"), with
#: E = 252 days converted to years on a 365-day year (the convention of the
#: paper's European-call draft, dt = E / (365 T)).
PAPER_POINT = dict(S0=127.62, K=130.0, r=0.00163, q=0.0163, sigma=0.2, expiry=252.0 / 365.0)


def option(model: int, S0: float, K: float, r: float, q: float, sigma: float, expiry: float,
           T: int) -> dict:
    return dict(model=int(model), S0=float(S0), K=float(K), r=float(r), q=float(q),
                sigma=float(sigma), expiry=float(expiry), T=int(T))


def draw_params(rng: np.random.Generator, model: int) -> dict:
    S0 = rng.uniform(50.0, 150.0)
    K = rng.uniform(50.0, 150.0)
    r = rng.uniform(0.01, 0.08)
    q = 0.0 if model == BSM_PUT else rng.uniform(0.01, 0.06)
    sigma = rng.uniform(0.1, 0.5)
    expiry = rng.uniform(0.25, 2.0)
    return dict(S0=S0, K=K, r=r, q=q, sigma=sigma, expiry=expiry)


def batch(config_id: int, log2T: int, n: int, model: int, T: int | None = None) -> list[dict]:
    """``n`` seeded options of one model at T = 2^log2T (or the given T)."""
    rng = np.random.default_rng([config_id, log2T])
    T = (1 << log2T) if T is None else T
    return [option(model, T=T, **draw_params(rng, model)) for _ in range(n)]


#: The single-option point used for the plain O(T^2) comparison (binomial).
CONFIG1 = option(BINOMIAL_CALL, 100.0, 100.0, 0.05, 0.03, 0.2, 1.0, 2000)


def serving_mix(n: int = 4096, seed=(5, 0), log2T_lo: float = 10.0, log2T_hi: float = 20.0):
    """Serving requests: model uniform over the three, T log-uniform in [2^lo, 2^hi]."""
    rng = np.random.default_rng(list(seed))
    out = []
    for _ in range(n):
        model = int(rng.integers(0, 3))
        T = int(round(2.0 ** rng.uniform(log2T_lo, log2T_hi)))
        out.append(option(model, T=max(T, 1), **draw_params(rng, model)))
    return out


def poisson_arrivals(n: int, rate_per_s: float, seed=(5, 1)) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process with the given rate."""
    rng = np.random.default_rng(list(seed))
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    return np.cumsum(gaps) - gaps[0]


def cells(opt: dict) -> float:
    """Equivalent lattice cells of one option, T^2 by convention for all models."""
    return float(opt["T"]) ** 2


def log2_ceil(x: int) -> int:
    return max(0, int(math.ceil(math.log2(max(1, x)))))
