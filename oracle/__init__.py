"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct FP64 reference for the three pricing problems
of Ahmad et al., "Fast American Option Pricing using Nonlinear Stencils"
(arXiv 2303.02317): the Theta(T^2) backward induction over the full binomial
lattice (Fig. 1, Definition 2.1), trinomial lattice (Sec. 3, appendix A.1) and
explicit finite-difference BSM grid (Sec. 4.2, eq. bsmG).  The arithmetic lives
in ``aop_oracle.c``; this module compiles it with gcc and calls it via ctypes.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library shares no code with it.

Parity status of each function (what pins it) is recorded in the test suite
``tests/test_oracle_pins.py``; every entry point here is pinned by brute force
at small T plus closed forms and identities fixed by the paper's formulas.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

BINOMIAL_CALL = 0
TRINOMIAL_CALL = 1
BSM_PUT = 2
MODEL_NAMES = {BINOMIAL_CALL: "binomial_call", TRINOMIAL_CALL: "trinomial_call", BSM_PUT: "bsm_put"}

DEFAULT_LAMBDA = 1.0 / 3.0  # dtau / ds^2 of the BSM grid
BOUNDARY_NONE_BSM = np.iinfo(np.int64).min

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "aop_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_handle = None


class OracleError(RuntimeError):
    pass


_STATUS = {0: "ok", 1: "invalid argument", 2: "probability/coefficient out of [0,1]", 3: "out of memory"}


def build(force: bool = False) -> str:
    """Compile ``liboracle.so`` in place with gcc (FP contraction off, portable ISA)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fPIC", "-shared",
               "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _declare(h):
    f = h.aop_oracle_price
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int] + [ctypes.c_double] * 6 + [ctypes.c_int64, ctypes.c_int,
                                                           ctypes.c_double,
                                                           ctypes.POINTER(ctypes.c_double),
                                                           ctypes.c_void_p, ctypes.c_void_p]
    return h


def _lib():
    global _handle
    with _lock:
        if _handle is None:
            if not os.path.exists(_LIB):
                build()
            _handle = _declare(ctypes.CDLL(_LIB))
    return _handle


def european_sum(model: int, S: float, K: float, r: float, q: float, sigma: float, expiry: float, T: int,
                 lib=None) -> float:
    """European call on the binomial or trinomial lattice as a sum over the
    binomial distribution of up moves (O(T); the trinomial lattice as 2T half
    steps), the closed form of the linear stencil applied T times."""
    lib = lib or _lib()
    f = lib.aop_oracle_european_sum
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int] + [ctypes.c_double] * 6 + [ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
    out = ctypes.c_double(0.0)
    rc = f(int(model), float(S), float(K), float(r), float(q), float(sigma), float(expiry), int(T), ctypes.byref(out))
    if rc != 0:
        raise OracleError("oracle rejected option: %s" % _STATUS.get(rc, rc))
    return out.value


GAUSS_WINDOW, GAUSS_SUM, GAUSS_ERF = 0, 1, 2


def european_gauss(method: int, S: float, K: float, r: float, q: float, sigma: float, expiry: float, T: int,
                   lib=None) -> float:
    """Gaussian approximations of the European binomial call: method 0 the
    O(sqrt T) windowed sum, 1 the O(T) sum, 2 the O(1) erf closed form."""
    lib = lib or _lib()
    f = lib.aop_oracle_european_gauss
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int] + [ctypes.c_double] * 6 + [ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
    out = ctypes.c_double(0.0)
    rc = f(int(method), float(S), float(K), float(r), float(q), float(sigma), float(expiry), int(T),
           ctypes.byref(out))
    if rc != 0:
        raise OracleError("oracle rejected option: %s" % _STATUS.get(rc, rc))
    return out.value


def load_variant(so_path: str):
    """Load another build of the oracle source (used by the mutation tests)."""
    return _declare(ctypes.CDLL(so_path))


def price(model: int, S: float, K: float, r: float, q: float, sigma: float, expiry: float,
          T: int, american: bool = True, lam: float = DEFAULT_LAMBDA,
          boundary: bool = False, margin: bool = False, lib=None, every: int | None = None):
    """Price one option by plain backward induction.

    ``every`` (binomial call only) overrides ``american``: 1 American, 0
    European, d >= 2 the Bermudan call exercisable on the rows i with
    (T - i) % d == 0 (every d steps back from expiry); its boundary on the
    other rows is the row's last column (every cell continues) and its margins
    there are NaN.

    Returns the price, or ``(price, boundary, margin)`` when either array is
    requested (``None`` for the one not requested).  ``boundary`` has T+1
    int64 entries: for the lattices the last continuation column of row i
    (-1 if none); for the BSM grid the last exercise offset k of step n
    (INT64_MIN if none).  ``margin`` has 2(T+1) entries: the decision gap at
    the boundary cell and at the next cell (units of K for the lattices,
    nondimensional for BSM), used to recognise near-ties.
    """
    lib = lib or _lib()
    out = ctypes.c_double(0.0)
    b = np.empty(T + 1, dtype=np.int64) if boundary else None
    mg = np.empty(2 * (T + 1), dtype=np.float64) if margin else None
    ex = (1 if american else 0) if every is None else int(every)
    rc = lib.aop_oracle_price(int(model), float(S), float(K), float(r), float(q), float(sigma),
                              float(expiry), int(T), ex, float(lam),
                              ctypes.byref(out),
                              b.ctypes.data if b is not None else None,
                              mg.ctypes.data if mg is not None else None)
    if rc != 0:
        raise OracleError("oracle rejected option: %s" % _STATUS.get(rc, rc))
    if boundary or margin:
        return out.value, b, mg
    return out.value


def price_option(opt: dict, **kw):
    """``price`` for an option dict with keys model, S0, K, r, q, sigma, expiry, T
    (and optionally european=True, or exercise_every=d for a Bermudan call)."""
    if opt.get("european") and "american" not in kw and "every" not in kw:
        kw = dict(kw, american=False)
    if opt.get("exercise_every", 1) != 1 and "every" not in kw:
        kw = dict(kw, every=int(opt["exercise_every"]))
    return price(opt["model"], opt["S0"], opt["K"], opt["r"], opt["q"], opt["sigma"],
                 opt["expiry"], opt["T"], **kw)


def price_many(opts, threads: int | None = None, **kw):
    """Price a list of option dicts, one option per host thread (ctypes drops the GIL)."""
    if threads is None:
        threads = len(os.sched_getaffinity(0))
    _lib()
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        return list(ex.map(lambda o: price_option(o, **kw), opts))
