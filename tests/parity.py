"""Shared parity criteria for GPU-vs-oracle comparisons (test code).

Prices: relative error <= rel_tol, or, for prices below 1e-3 K (where the
FFT's normwise error dominates the relative error of a tiny value), absolute
error <= abs_tol_k * K.

Boundaries: where floating point decides an integer, both sides take the
decision in FP64 but with differently rounded continuation values (direct sums
vs FFT correlation), so an index may differ by one where the oracle's own
decision margin is below ``tie`` (in units of K for the lattices, of the
nondimensional value for BSM).  Any other difference is a failure.
"""
import numpy as np

REL_FP64 = 1e-9
ABS_FP64_K = 1e-13
REL_MIXED = 1e-6
ABS_MIXED_K = 1e-9
TIE = 1e-9
BSM_NONE = int(np.iinfo(np.int64).min)


def price_ok(got, ref, K, rel_tol=REL_FP64, abs_tol_k=ABS_FP64_K):
    if not np.isfinite(got):
        return False
    err = abs(got - ref)
    if err <= rel_tol * abs(ref):
        return True
    return abs(ref) < 1e-3 * K and err <= abs_tol_k * K


def price_errors(got, ref):
    err = abs(got - ref)
    return err, err / max(abs(ref), 1e-300)


def golden_margins(rec):
    """Decision margins stored with a golden record (see tests/golden/make_golden.py),
    flattened as the oracle returns them (2 per sampled row), or None."""
    if "margin" not in rec:
        return None
    conv = {None: np.nan, "inf": np.inf, "-inf": -np.inf}
    return np.array([conv[v] if v is None or isinstance(v, str) else float(v)
                     for pair in rec["margin"] for v in pair], dtype=np.float64)


def boundary_mismatches(gb, ob, margin, model, T):
    """Rows where the GPU boundary differs from the oracle's other than by a near-tie.

    The BSM sentinel INT64_MIN ("no exercise cell") only ever equals itself:
    indices are compared as Python integers, so no difference overflows."""
    bad = []
    rows = np.nonzero(np.asarray(gb) != np.asarray(ob))[0]
    for i in rows:
        g, o = int(gb[i]), int(ob[i])
        if model == 2 and (g == np.iinfo(np.int64).min or o == np.iinfo(np.int64).min):
            bad.append((int(i), g, o))
            continue
        if abs(g - o) != 1:
            bad.append((int(i), g, o))
            continue
        m = margin[2 * i] if g < o else margin[2 * i + 1]
        if not (np.isfinite(m) and abs(m) <= TIE):
            bad.append((int(i), g, o))
    return bad
