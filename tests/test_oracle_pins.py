"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Every check here compares the oracle with something other than itself: brute
force on tiny trees, closed-form sums, identities implied by the paper's
formulas, Black-Scholes limits, high-precision arithmetic, and the lemmas of
Sec. 2.2 / appendix A.2 / Sec. 4.2 about the red-green divider.  A plausible
mistake in the oracle (swapped child weights, a wrong exponent index, a dropped
drift term, the wrong tie rule) fails at least one of them.
"""
import math

import mpmath

import numpy as np
import pytest

from paper_2303_02317_amd import inputs
from tests import pins

B, TR, P = 0, 1, 2  # model ids


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


# ------------------------------------------------------------ brute force
PARAMS_SMALL = [
    (100.0, 100.0, 0.05, 0.03, 0.2, 1.0),
    (120.0, 100.0, 0.08, 0.06, 0.3, 1.5),   # in the money, q > r: early exercise
    (80.0, 110.0, 0.02, 0.05, 0.45, 0.5),
    (140.0, 60.0, 0.01, 0.06, 0.1, 2.0),    # deep ITM: exercise at the root
]


@pytest.mark.parametrize("prm", PARAMS_SMALL)
@pytest.mark.parametrize("T", [1, 2, 3, 7, 12])
def test_binomial_vs_brute_force_tree(oracle_mod, prm, T):
    S, K, r, q, s, E = prm
    for am in (True, False):
        got = oracle_mod.price(B, S, K, r, q, s, E, T, american=am)
        ref = pins.brute_binomial(S, K, r, q, s, E, T, american=am)
        assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref))


@pytest.mark.parametrize("prm", PARAMS_SMALL)
@pytest.mark.parametrize("T", [1, 2, 4, 7])
def test_trinomial_vs_brute_force_tree(oracle_mod, prm, T):
    S, K, r, q, s, E = prm
    for am in (True, False):
        got = oracle_mod.price(TR, S, K, r, q, s, E, T, american=am)
        ref = pins.brute_trinomial(S, K, r, q, s, E, T, american=am)
        assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref))


@pytest.mark.parametrize("prm", [(100.0, 100.0, 0.05, 0.2, 1.0), (90.0, 110.0, 0.08, 0.45, 2.0),
                                 (130.0, 70.0, 0.01, 0.1, 0.25), (60.0, 140.0, 0.06, 0.3, 1.0)])
@pytest.mark.parametrize("T", [1, 2, 5, 8])
def test_bsm_put_vs_brute_force_paths(oracle_mod, prm, T):
    S, K, r, s, E = prm
    for am in (True, False):
        got = oracle_mod.price(P, S, K, r, 0.0, s, E, T, american=am)
        ref = pins.brute_bsm_put(S, K, r, s, E, T, american=am)
        assert abs(got - ref) <= 1e-13 * K


def test_binomial_high_precision(oracle_mod):
    # Rounding of the FP64 induction stays at the 1e-13 level (mpmath, 50 digits).
    for prm in PARAMS_SMALL:
        S, K, r, q, s, E = prm
        got = oracle_mod.price(B, S, K, r, q, s, E, 96)
        ref = pins.mp_binomial(S, K, r, q, s, E, 96)
        assert abs(got - ref) <= 1e-13 * max(1.0, ref)


# ------------------------------------------------------ linear-part pins
@pytest.mark.parametrize("T", [50, 333, 2000])
def test_european_binomial_closed_form_sum(oracle_mod, T):
    rng = np.random.default_rng([101, T])
    for _ in range(4):
        p = inputs.draw_params(rng, B)
        got = oracle_mod.price(B, p["S0"], p["K"], p["r"], p["q"], p["sigma"], p["expiry"], T,
                               american=False)
        ref = pins.european_binomial_sum(p["S0"], p["K"], p["r"], p["q"], p["sigma"], p["expiry"], T)
        assert abs(got - ref) <= 1e-11 * max(ref, 1e-3 * p["K"])


def test_forward_identity(oracle_mod):
    # s0/u + s1 u = e^{-Y dt} (Lemma 2.2 proof): with every leaf in the money the
    # European lattice value is exactly S e^{-qE} - K e^{-rE}.  The swapped
    # weight orientation misses this by tens of percent.
    S, r, q, s, E, T = 120.0, 0.08, 0.01, 0.2, 1.0, 1000
    K = 0.5 * S * math.exp(-s * math.sqrt(E * T))  # below the lowest leaf
    got = oracle_mod.price(B, S, K, r, q, s, E, T, american=False)
    exact = S * math.exp(-q * E) - K * math.exp(-r * E)
    assert rel(got, exact) <= 1e-12
    # Trinomial: s_d/u + s_o + s_u u = e^{-Y dt} likewise.
    K = 0.5 * S * math.exp(-s * math.sqrt(2 * E * T))
    got = oracle_mod.price(TR, S, K, r, q, s, E, T, american=False)
    exact = S * math.exp(-q * E) - K * math.exp(-r * E)
    assert rel(got, exact) <= 1e-12


@pytest.mark.parametrize("T", [10, 250, 777])
def test_european_trinomial_equals_binomial_2T(oracle_mod, T):
    # p_u = alpha^2, p_d = (1-alpha)^2 with alpha the binomial p at dt/2 (Sec. 3),
    # so one trinomial step is two binomial steps: TOPM(T) == BOPM(2T) (European).
    rng = np.random.default_rng([102, T])
    for _ in range(3):
        p = inputs.draw_params(rng, B)
        a = oracle_mod.price(TR, p["S0"], p["K"], p["r"], p["q"], p["sigma"], p["expiry"], T,
                             american=False)
        b = oracle_mod.price(B, p["S0"], p["K"], p["r"], p["q"], p["sigma"], p["expiry"], 2 * T,
                             american=False)
        assert abs(a - b) <= 1e-11 * max(b, 1e-3 * p["K"])


@pytest.mark.parametrize("T", [3, 40, 150])
def test_european_bsm_multinomial_expansion(oracle_mod, T):
    rng = np.random.default_rng([103, T])
    for _ in range(3):
        p = inputs.draw_params(rng, P)
        got = oracle_mod.price(P, p["S0"], p["K"], p["r"], 0.0, p["sigma"], p["expiry"], T,
                               american=False)
        ref = pins.european_bsm_multinomial(p["S0"], p["K"], p["r"], p["sigma"], p["expiry"], T)
        assert abs(got - ref) <= 1e-11 * p["K"]


def test_continuous_limits(oracle_mod):
    # The lattices and the explicit scheme converge to the Black-Scholes values.
    S, K, r, q, s, E = 100.0, 100.0, 0.05, 0.03, 0.2, 1.0
    bs = pins.bs_call_div(S, K, r, q, s, E)
    for T, tol in ((250, 1e-2), (2000, 1.5e-3), (8000, 4e-4)):
        assert abs(oracle_mod.price(B, S, K, r, q, s, E, T, american=False) - bs) <= tol
    assert abs(oracle_mod.price(TR, S, K, r, q, s, E, 2000, american=False) - bs) <= 1e-3
    for (S, K) in ((100.0, 110.0), (120.0, 100.0)):
        bp = pins.bs_put(S, K, 0.05, 0.25, 1.0)
        for T in (500, 2000):
            assert abs(oracle_mod.price(P, S, K, 0.05, 0.0, 0.25, 1.0, T, american=False) - bp) <= 2e-3 * K


# --------------------------------------------------------- American facts
def test_no_dividend_call_is_european(oracle_mod):
    # Y = 0: Lemma 2.3 leaves no green cell, so the American call is European.
    for T in (100, 2000):
        for model in (B, TR):
            a = oracle_mod.price(model, 100.0, 90.0, 0.05, 0.0, 0.3, 1.0, T)
            e = oracle_mod.price(model, 100.0, 90.0, 0.05, 0.0, 0.3, 1.0, T, american=False)
            assert rel(a, e) <= 1e-14


def test_bounds_and_monotonicity(oracle_mod):
    rng = np.random.default_rng([104, 0])
    T = 300
    for model in (B, TR, P):
        for _ in range(8):
            p = inputs.draw_params(rng, model)
            args = (p["S0"], p["K"], p["r"], p["q"], p["sigma"], p["expiry"], T)
            am = oracle_mod.price(model, *args)
            eu = oracle_mod.price(model, *args, american=False)
            intrinsic = (p["S0"] - p["K"]) if model != P else (p["K"] - p["S0"])
            assert am >= eu - 1e-13 * p["K"]
            assert am >= intrinsic - 1e-12 * p["K"]
            assert am >= 0.0
            # strike monotonicity (exact: lattice nodes do not move with K)
            up = oracle_mod.price(model, p["S0"], p["K"] * 1.01, *args[2:])
            if model == P:
                assert up >= am
                assert am <= p["K"]  # v in [0,1] (maximum principle for a,b,c >= 0)
            else:
                assert up <= am
            # volatility monotonicity (observed, not proven for fixed T)
            hv = oracle_mod.price(model, p["S0"], p["K"], p["r"], p["q"], p["sigma"] * 1.05,
                                  p["expiry"], T)
            assert hv >= am - 1e-12 * p["K"]


def test_paper_parameter_point(oracle_mod):
    # The experiment point of Sec. 5 (E read in days / 365): sane prices.
    pp = inputs.PAPER_POINT
    for model in (B, TR):
        am = oracle_mod.price(model, pp["S0"], pp["K"], pp["r"], pp["q"], pp["sigma"], pp["expiry"], 1024)
        eu = oracle_mod.price(model, pp["S0"], pp["K"], pp["r"], pp["q"], pp["sigma"], pp["expiry"], 1024,
                              american=False)
        bs = pins.bs_call_div(pp["S0"], pp["K"], pp["r"], pp["q"], pp["sigma"], pp["expiry"])
        assert am >= eu and abs(eu - bs) < 2e-2


# ---------------------------------------------------- the divider's lemmas
def _near_tie(m, idx):
    return np.isfinite(m[idx]) and abs(m[idx]) < 1e-12


def test_binomial_divider_lemmas_on_full_grid():
    # Lemma 2.2 (right of green is green), Lemma 2.4 (below green is green),
    # Lemma 2.5 (time decay G_{i,j} >= G_{i+2,j+1}) and the corollary's
    # contiguous red prefix, checked on full numpy grids.
    rng = np.random.default_rng([105, 0])
    for _ in range(6):
        p = inputs.draw_params(rng, B)
        T = 160
        G, red = pins.grid_binomial(p["S0"], p["K"], p["r"], p["q"], p["sigma"], p["expiry"], T)
        for i in range(T + 1):
            rr = red[i, :i + 1]
            nred = int(rr.sum())
            assert rr[:nred].all(), "red cells of a row form a prefix"
        for i in range(T - 1):
            for j in range(i + 1):
                if not red[i + 1, j]:
                    assert not red[i, j], "below a green cell is green"
        for i in range(T - 1):
            for j in range(i):
                assert G[i, j] >= G[i + 2, j + 1] - 1e-12 * p["K"]


@pytest.mark.parametrize("model", [B, TR])
def test_lattice_boundary_moves_at_most_one(oracle_mod, model):
    rng = np.random.default_rng([106, model])
    T = 1500
    for _ in range(8):
        p = inputs.draw_params(rng, model)
        pr, b, mg = oracle_mod.price(model, p["S0"], p["K"], p["r"], p["q"], p["sigma"],
                                     p["expiry"], T, boundary=True, margin=True)
        width = (lambda i: i) if model == B else (lambda i: 2 * i)
        for i in range(T - 1):
            if b[i + 1] < 0 or b[i + 1] == width(i + 1):
                continue  # no red cell, or an all-red row (no divider)
            ok = b[i + 1] - 1 <= b[i] <= b[i + 1]
            if not ok:
                assert _near_tie(mg, 2 * i) or _near_tie(mg, 2 * i + 1)
        # Lemma 2.3 (range of green), binomial only: the first green column
        # j = b_i + 1 satisfies j >= i/2 + ln(K/S (1-e^{-R dt})/(1-e^{-Y dt}))/(2 V sqrt(dt)).
        if model == B:
            dt = p["expiry"] / T
            bound_c = math.log(p["K"] / p["S0"] * (1 - math.exp(-p["r"] * dt)) /
                               (1 - math.exp(-p["q"] * dt))) / (2 * p["sigma"] * math.sqrt(dt))
            for i in range(T):
                j = b[i] + 1
                if j <= i:
                    assert j >= i / 2 + bound_c - 1e-9


def test_bsm_boundary_moves_at_most_one(oracle_mod):
    # Theorem 4.2: 0 <= k_n - k_{n+1} <= 1 when a, b, c >= 0.
    rng = np.random.default_rng([107, 0])
    T = 1500
    nmin = 64
    for _ in range(8):
        p = inputs.draw_params(rng, P)
        pr, b, mg = oracle_mod.price(P, p["S0"], p["K"], p["r"], 0.0, p["sigma"], p["expiry"], T,
                                     boundary=True, margin=True)
        none = np.iinfo(np.int64).min
        for n in range(1, T):
            if b[n] == none or b[n + 1] == none or b[n] >= T - n:
                continue
            if not (0 <= b[n] - b[n + 1] <= 1):
                assert _near_tie(mg, 2 * (n + 1)) or _near_tie(mg, 2 * (n + 1) + 1) or n < nmin


def test_rejections(oracle_mod):
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.price(P, 100, 100, 0.05, 0.02, 0.2, 1.0, 100)  # q != 0 for BSM
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.price(B, -1, 100, 0.05, 0.02, 0.2, 1.0, 100)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.price(B, 100, 100, 0.9, 0.0, 0.01, 1.0, 1)  # p > 1


def test_tie_rule_is_red(oracle_mod):
    # Definition 2.1: a cell is red when G^red >= G^green.  With S = K and T
    # even, the expiry cell j = T/2 has G^red = 0 = G^green, so it is red and
    # the expiry row's boundary is exactly T/2.
    for T in (2, 200, 2000):
        _, b, mg = oracle_mod.price(B, 100.0, 100.0, 0.05, 0.03, 0.2, 1.0, T, boundary=True, margin=True)
        assert b[T] == T // 2 and mg[2 * T] == 0.0


# ------------------------------------------------- non-finite guard (overflow)
OVERFLOW = [
    # sigma sqrt(E T) > 709.8: the top of the lattice overflows to +inf in FP64
    (100.0, 100.0, 0.05, 0.03, 80.0, 1.0, 96),
    (120.0, 90.0, 0.06, 0.02, 60.0, 1.5, 120),
    (100.0, 100.0, 0.05, 0.0, 80.0, 1.0, 96),   # q = 0: no exercise in exact arithmetic
    (100.0, 100.0, 0.03, 0.06, 75.0, 1.0, 100),
]


@pytest.mark.parametrize("prm", OVERFLOW)
def test_overflowing_lattice_against_high_precision(oracle_mod, prm):
    # Cells whose exercise value overflows are exercise cells (the guard of
    # Definition 2.1's red test).  They lie where the risk-neutral weight of
    # reaching them is far below 1e-300, so the FP64 price still equals the
    # exact lattice value; without the guard inf >= inf marks them red and the
    # infinity reaches the root.
    S, K, r, q, s, E, T = prm
    assert s * math.sqrt(E * T) > 709.8
    for model, ref in ((B, pins.mp_binomial), (TR, pins.mp_trinomial)):
        exact = ref(S, K, r, q, s, E, T)
        got = oracle_mod.price(model, S, K, r, q, s, E, T)
        got_m, _, _ = oracle_mod.price(model, S, K, r, q, s, E, T, boundary=True, margin=True)
        assert math.isfinite(got) and abs(got - exact) <= 1e-13 * exact
        assert got_m == got


def test_trinomial_high_precision(oracle_mod):
    for prm in PARAMS_SMALL:
        S, K, r, q, s, E = prm
        got = oracle_mod.price(TR, S, K, r, q, s, E, 60)
        ref = pins.mp_trinomial(S, K, r, q, s, E, 60)
        assert abs(got - ref) <= 1e-13 * max(1.0, ref)


# ------------------------------------------------ negative rate, no dividend
@pytest.mark.parametrize("model", [B, TR])
def test_negative_rate_no_dividend_exercises(oracle_mod, model):
    # With R < 0 and Y = 0 the no-exercise lemma (which needs R > 0) does not
    # apply: deep in the money, exercising now beats holding.  Brute force on
    # small trees and the immediate-exercise value pin the oracle there.
    prm = (150.0, 60.0, -0.03, 0.0, 0.15, 2.0)
    brute = pins.brute_binomial if model == B else pins.brute_trinomial
    for T in (5, 8):
        got = oracle_mod.price(model, *prm, T)
        assert abs(got - brute(*prm, T)) <= 1e-12 * got
    am = oracle_mod.price(model, *prm, 400)
    eu = oracle_mod.price(model, *prm, 400, american=False)
    assert am == pytest.approx(150.0 - 60.0, abs=1e-12) and eu < am - 1.0


# ------------------------------------------------------ boundary references
BPRM = [
    (120.0, 100.0, 0.08, 0.06, 0.3, 1.5),
    (100.0, 100.0, 0.05, 0.03, 0.2, 1.0),
    (140.0, 60.0, 0.01, 0.06, 0.1, 2.0),
    (90.0, 105.0, 0.02, 0.05, 0.45, 0.5),
]


def _cmp_rows(got, ref, skip=()):
    bad = [(i, int(got[i]), ref[i]) for i in range(len(ref)) if i not in skip and ref[i] != "tie"
           and int(got[i]) != ref[i]]
    assert not bad, bad[:5]


@pytest.mark.parametrize("prm", BPRM)
def test_lattice_boundary_against_brute_force_decisions(oracle_mod, prm):
    # Each node's red/green decision recorded along every path of a
    # non-recombining tree gives every row's boundary independently of the
    # oracle's in-place sweep.
    for T in (4, 9, 11):
        _, ref = pins.brute_binomial_boundary(*prm, T)
        _, b, _ = oracle_mod.price(B, *prm, T, boundary=True)
        _cmp_rows(b, ref)
    for T in (3, 6):
        _, ref = pins.brute_trinomial_boundary(*prm, T)
        _, b, _ = oracle_mod.price(TR, *prm, T, boundary=True)
        _cmp_rows(b, ref)


@pytest.mark.parametrize("prm", [(90.0, 110.0, 0.08, 0.45, 2.0), (100.0, 100.0, 0.05, 0.2, 1.0),
                                 (60.0, 140.0, 0.06, 0.3, 1.0), (70.0, 80.0, 0.07, 0.15, 2.0)])
def test_bsm_boundary_against_brute_force_decisions(oracle_mod, prm):
    S, K, r, s, E = prm
    none = np.iinfo(np.int64).min
    for T in (3, 6, 8):
        _, ref = pins.brute_bsm_put_boundary(S, K, r, s, E, T)
        _, b, _ = oracle_mod.price(P, S, K, r, 0.0, s, E, T, boundary=True)
        ref = [none if x is None else x for x in ref]
        _cmp_rows(b, ref)


@pytest.mark.parametrize("model", [TR, P])
def test_boundary_against_full_numpy_grid(oracle_mod, model):
    # The oracle's recorded boundary equals the last red column (lattices) or
    # last exercise offset (BSM) of a full numpy grid, row by row.
    rng = np.random.default_rng([108, model])
    T = 200
    for _ in range(5):
        p = inputs.draw_params(rng, model)
        _, b, mg = oracle_mod.price(model, p["S0"], p["K"], p["r"], p["q"], p["sigma"], p["expiry"], T,
                                    boundary=True, margin=True)
        if model == TR:
            G, red = pins.grid_trinomial(p["S0"], p["K"], p["r"], p["q"], p["sigma"], p["expiry"], T)
            for i in range(T + 1):
                reds = np.nonzero(red[i, :2 * i + 1])[0]
                ref = int(reds.max()) if reds.size else -1
                if b[i] != ref:
                    assert _near_tie(mg, 2 * i) or _near_tie(mg, 2 * i + 1), (i, b[i], ref)
        else:
            V, green = pins.grid_bsm_put(p["S0"], p["K"], p["r"], p["sigma"], p["expiry"], T)
            for n in range(T + 1):
                gs = np.nonzero(green[n])[0]
                ref = int(gs.max()) - T if gs.size else np.iinfo(np.int64).min
                if b[n] != ref:
                    assert _near_tie(mg, 2 * n) or _near_tie(mg, 2 * n + 1), (n, b[n], ref)


def test_binomial_boundary_against_full_numpy_grid(oracle_mod):
    rng = np.random.default_rng([108, B])
    T = 240
    for _ in range(5):
        p = inputs.draw_params(rng, B)
        _, b, mg = oracle_mod.price(B, p["S0"], p["K"], p["r"], p["q"], p["sigma"], p["expiry"], T,
                                    boundary=True, margin=True)
        G, red = pins.grid_binomial(p["S0"], p["K"], p["r"], p["q"], p["sigma"], p["expiry"], T)
        for i in range(T + 1):
            reds = np.nonzero(red[i, :i + 1])[0]
            ref = int(reds.max()) if reds.size else -1
            if b[i] != ref:
                assert _near_tie(mg, 2 * i) or _near_tie(mg, 2 * i + 1), (i, b[i], ref)


# ---------------------------------------------- survey-time cross-check values
def test_survey_cross_check_values(oracle_mod):
    # Values computed independently (throwaway numpy) when the path was
    # surveyed, at the single-option point (S = K = 100, R = 0.05, Y = 0.03,
    # V = 0.2, E = 1 year) unless stated.
    cfg1 = (100.0, 100.0, 0.05, 0.03, 0.2, 1.0)
    p, b, _ = oracle_mod.price(B, *cfg1, 2000, boundary=True)
    assert p == pytest.approx(8.65179401413394, rel=1e-13)
    assert list(b[:6]) == [0, 1, 2, 3, 4, 5] and b[1998] == 1056 and b[1999] == 1056 and b[2000] == 1000
    assert oracle_mod.price(B, *cfg1, 2000, american=False) == pytest.approx(8.65156725043792, rel=1e-13)
    p, b, _ = oracle_mod.price(TR, *cfg1, 2000, boundary=True)
    assert p == pytest.approx(8.65227509654429, rel=1e-13) and b[1999] == 2079
    assert oracle_mod.price(TR, *cfg1, 2000, american=False) == pytest.approx(8.65204788716948, rel=1e-13)
    bsm = (100.0, 100.0, 0.05, 0.0, 0.2, 1.0)
    assert oracle_mod.price(P, *bsm, 2000) == pytest.approx(6.09033225614848, rel=1e-13)
    assert oracle_mod.price(P, *bsm, 2000, american=False) == pytest.approx(5.57329504835891, rel=1e-13)
    for T, v in ((1, 10.53727992187781), (2, 7.777507797933374), (5, 9.033635181083387),
                 (12, 8.494212397930681)):
        assert oracle_mod.price(B, *cfg1, T) == pytest.approx(v, rel=1e-14)
    d = (oracle_mod.price(TR, 110.0, 100.0, 0.08, 0.02, 0.3, 1.5, 500, american=False) -
         oracle_mod.price(B, 110.0, 100.0, 0.08, 0.02, 0.3, 1.5, 1000, american=False))
    assert abs(d) <= 1e-11


def test_binomial_margins_against_full_numpy_grid(oracle_mod):
    # The decision gaps the oracle records (used to recognise near-ties in the
    # parity tests) are (c - e)/K at the last red cell and (e - c)/K at the
    # cell after it, with c the continuation value of Definition 2.1 computed
    # from the row below on a full numpy grid.
    rng = np.random.default_rng([109, B])
    T = 240
    for _ in range(4):
        p = inputs.draw_params(rng, B)
        S, K = p["S0"], p["K"]
        _, b, mg = oracle_mod.price(B, S, K, p["r"], p["q"], p["sigma"], p["expiry"], T,
                                    boundary=True, margin=True)
        G, _ = pins.grid_binomial(S, K, p["r"], p["q"], p["sigma"], p["expiry"], T)
        _, u, _, pp, m = pins.bopm_params(p["r"], p["q"], p["sigma"], p["expiry"], T)
        for i in range(T):
            j = np.arange(i + 1)
            c = m * (1 - pp) * G[i + 1, :i + 1] + m * pp * G[i + 1, 1:i + 2]
            gap = (c - (S * u ** (2.0 * j - i) - K)) / K
            last = int(b[i])
            if last >= 0:
                assert abs(mg[2 * i] - gap[last]) <= 1e-12, (i, mg[2 * i], gap[last])
            else:
                assert np.isnan(mg[2 * i])
            if last + 1 <= i:
                assert abs(mg[2 * i + 1] + gap[last + 1]) <= 1e-12, (i, mg[2 * i + 1], -gap[last + 1])
            else:
                assert np.isnan(mg[2 * i + 1])


def test_trinomial_negative_rate_breaks_step_bound(oracle_mod):
    # Why the library rejects a trinomial call with R < 0: the decomposition
    # needs the boundary to drop by at most two columns per row (the cone of a
    # trinomial cell widens by two per row), which the lemmas of Sec. 3 give
    # for R >= 0.  With R < 0 and Y = 0 the oracle shows drops of three or
    # more; the binomial lattice keeps its one-column bound on the same inputs.
    prm = (88.04753706433236, 121.32578641244521, -0.038748219583468815, 0.0, 0.4966706867960785,
           1.5164334456388935)
    T = 1000
    _, b, _ = oracle_mod.price(TR, *prm, T, boundary=True)
    drops = [int(b[i + 1] - b[i]) for i in range(T - 1) if b[i + 1] >= 0]
    assert max(drops) > 2
    _, b, _ = oracle_mod.price(B, *prm, T, boundary=True)
    assert max(int(b[i + 1] - b[i]) for i in range(T - 1) if b[i + 1] >= 0) <= 1
    # with R >= 0 and a dividend the trinomial bound holds on the same spot,
    # strike and volatility (with Y = 0 and R >= 0 nothing exercises below the
    # expiry row in exact arithmetic, and the library prices that case as one
    # correlation without a boundary)
    for r in (0.0, 0.02):
        _, b, _ = oracle_mod.price(TR, prm[0], prm[1], r, 0.02, prm[4], prm[5], T, boundary=True)
        assert max(int(b[i + 1] - b[i]) for i in range(T - 1) if b[i + 1] >= 0) <= 2


# ------------------------------------------ European closed-form lattice sums
@pytest.mark.parametrize("model", [B, TR])
def test_european_sum_equals_lattice_induction(oracle_mod, model):
    # The O(T) sum over the up-move distribution equals the plain induction
    # without exercise (the linear stencil applied T times) for both lattices.
    rng = np.random.default_rng([110, model])
    for T in (1, 2, 3, 17, 256, 2048):
        for _ in range(4):
            p = inputs.draw_params(rng, model)
            args = (p["S0"], p["K"], p["r"], p["q"], p["sigma"], p["expiry"], T)
            got = oracle_mod.european_sum(model, *args)
            ref = oracle_mod.price(model, *args, american=False)
            assert abs(got - ref) <= 1e-12 * max(ref, 1e-3 * p["K"]), (T, got, ref)


@pytest.mark.parametrize("model", [B, TR])
def test_european_sum_against_high_precision(oracle_mod, model):
    # 40-digit binomial sums (trinomial: its own three-way path sum) at T where
    # the recurrence runs a few thousand terms from the mode.
    with mpmath.workdps(40):
        for (S, K, r, q, s, E, T) in ((100.0, 95.0, 0.05, 0.02, 0.3, 1.2, 3000), (80.0, 120.0, 0.03, 0.01, 0.45, 2.0, 1500)):
            got = oracle_mod.european_sum(model, S, K, r, q, s, E, T)
            if model == B:
                _, u, _, p, m = pins.bopm_params(r, q, s, E, T)
                mp_ = mpmath.mpf
                dt = mp_(E) / T
                a = mp_(s) * mpmath.sqrt(dt)
                uu = mpmath.e ** a
                pp = (mpmath.e ** ((mp_(r) - q) * dt) - 1 / uu) / (uu - 1 / uu)
                tot = mp_(0)
                for k in range(T + 1):
                    x = S * mpmath.e ** ((2 * k - T) * a)
                    if x > K:
                        tot += mpmath.binomial(T, k) * pp ** k * (1 - pp) ** (T - k) * (x - K)
                exact = tot * mpmath.e ** (-mp_(r) * E)
            else:
                exact = pins.mp_trinomial(S, K, r, q, s, E, min(T, 400), american=False)
                got = oracle_mod.european_sum(model, S, K, r, q, s, E, min(T, 400))
            assert abs(got - float(exact)) <= 1e-12 * float(exact), (got, exact)


# ------------------------------- Gaussian / erf European approximations
GP = [(100.0, 95.0, 0.05, 0.02, 0.3, 1.2), (80.0, 120.0, 0.03, 0.01, 0.45, 2.0), (130.0, 70.0, 0.07, 0.05, 0.15, 0.5)]


@pytest.mark.parametrize("prm", GP)
def test_gauss_erf_form_is_the_integral(oracle_mod, prm):
    # The O(1) form is the closed-form integral of the same Gaussian-weighted
    # payoff from ceil(T/2 + ln(K/S)/(2 ln u)) to T: checked by quadrature.
    from scipy import integrate

    S, K, r, q, s, E = prm
    for T in (64, 1000, 50000):
        dt, u, _, p, m = pins.bopm_params(r, q, s, E, T)
        mu, v, lu = p * T, p * (1 - p) * T, math.log(u)
        x0 = math.ceil(T / 2 + math.log(K / S) / (2 * lu))
        f = lambda x: (S * math.exp((2 * x - T) * lu) - K) * math.exp(-(x - mu) ** 2 / (2 * v))
        lo = min(x0, T)
        pts = [c for c in (mu - 8 * math.sqrt(v), mu, mu + 8 * math.sqrt(v)) if lo < c < T]
        val, _ = integrate.quad(f, lo, T, points=pts or None, limit=400, epsabs=0, epsrel=1e-13)
        ref = m ** T * val / math.sqrt(2 * math.pi * v)
        got = oracle_mod.european_gauss(oracle_mod.GAUSS_ERF, S, K, r, q, s, E, T)
        assert abs(got - ref) <= 1e-9 * max(abs(ref), 1e-3 * K), (T, got, ref)


@pytest.mark.parametrize("prm", GP)
def test_gauss_sums_approximate_the_lattice(oracle_mod, prm):
    # The normal approximation of the up-move count is a local limit theorem:
    # its sums approach the exact binomial sum with an error of order 1/T
    # (a wrong mean, variance or discount would not converge at all), and as
    # T grows all three forms approach Black-Scholes with a dividend yield.
    S, K, r, q, s, E = prm
    errs = []
    for T in (1000, 10000, 100000):
        ex = oracle_mod.european_sum(0, S, K, r, q, s, E, T)
        full = oracle_mod.european_gauss(oracle_mod.GAUSS_SUM, S, K, r, q, s, E, T)
        errs.append(abs(full - ex) / ex)
    assert errs[0] < 2e-3
    assert 4.0 < errs[0] / errs[1] < 25.0 and 4.0 < errs[1] / errs[2] < 25.0, errs
    T = 1 << 20
    bs = pins.bs_call_div(S, K, r, q, s, E)
    for meth in (oracle_mod.GAUSS_WINDOW, oracle_mod.GAUSS_SUM, oracle_mod.GAUSS_ERF):
        assert abs(oracle_mod.european_gauss(meth, S, K, r, q, s, E, T) - bs) <= 2e-3 * bs


def test_gauss_window_covers_the_mass(oracle_mod):
    # The O(sqrt T) window is the full sum cut at 6 standard deviations: equal
    # to it when the window spans every x, and within the Gaussian tail beyond
    # 6 sd otherwise.
    S, K, r, q, s, E = GP[0]
    for T in (8, 16, 30):  # mu +- 6 sd covers [0, T-1]
        w = oracle_mod.european_gauss(oracle_mod.GAUSS_WINDOW, S, K, r, q, s, E, T)
        f = oracle_mod.european_gauss(oracle_mod.GAUSS_SUM, S, K, r, q, s, E, T)
        assert w == f
    for T in (4096, 1 << 20):
        w = oracle_mod.european_gauss(oracle_mod.GAUSS_WINDOW, S, K, r, q, s, E, T)
        f = oracle_mod.european_gauss(oracle_mod.GAUSS_SUM, S, K, r, q, s, E, T)
        assert 0 <= f - w <= 1e-6 * f


# ----------------------------------------------- Bermudan (discrete exercise)
@pytest.mark.parametrize("every", [2, 3, 5])
def test_bermudan_against_brute_force(oracle_mod, every):
    prm = (120.0, 100.0, 0.08, 0.06, 0.3, 1.5)
    for T in (5, 9, 12):
        got = oracle_mod.price(B, *prm, T, every=every)
        assert abs(got - pins.brute_binomial_bermudan(*prm, T, every)) <= 1e-12 * prm[1]


def test_bermudan_limits_and_ordering(oracle_mod):
    rng = np.random.default_rng([111, 0])
    for _ in range(6):
        p = inputs.draw_params(rng, B)
        args = (p["S0"], p["K"], p["r"], p["q"], p["sigma"], p["expiry"], 600)
        am = oracle_mod.price(B, *args)
        eu = oracle_mod.price(B, *args, american=False)
        assert oracle_mod.price(B, *args, every=1) == am
        assert oracle_mod.price(B, *args, every=601) == eu
        vals = [oracle_mod.price(B, *args, every=d) for d in (1, 2, 4, 8, 600)]
        # nested exercise sets: more exercise dates never lower the value
        assert all(vals[k] >= vals[k + 1] - 1e-12 * p["K"] for k in range(len(vals) - 1))
        assert vals[-1] >= eu - 1e-12 * p["K"]


def test_trinomial_is_bermudan_binomial_on_twice_the_steps(oracle_mod):
    # Sec. 3's trinomial lattice with p_u = alpha^2, p_o = 2 alpha (1 - alpha),
    # p_d = (1 - alpha)^2 is the binomial lattice of 2T steps with up
    # probability alpha, exercisable every second row: same price, and the
    # trinomial boundary of row i is the binomial boundary of row 2i.
    rng = np.random.default_rng([112, 0])
    for _ in range(5):
        p = inputs.draw_params(rng, TR)
        T = 300
        args = (p["S0"], p["K"], p["r"], p["q"], p["sigma"], p["expiry"])
        pt, bt, mt = oracle_mod.price(TR, *args, T, boundary=True, margin=True)
        pb, bb, mb = oracle_mod.price(B, *args, 2 * T, boundary=True, margin=True, every=2)
        assert abs(pt - pb) <= 1e-11 * max(pt, 1e-3 * p["K"])
        for i in range(T):
            if bt[i] != bb[2 * i]:
                assert _near_tie(mt, 2 * i) or _near_tie(mt, 2 * i + 1), (i, bt[i], bb[2 * i])


@pytest.mark.parametrize("every", [2, 3, 8, 32])
def test_bermudan_boundary_drops_at_most_one_column_per_row(oracle_mod, every):
    # The reading the decomposition of a Bermudan call rests on: between two
    # exercise rows i and i - d the boundary drops by at most d columns (one
    # per row, as Corollary 2.6 gives on every row of the American lattice),
    # so cells left of b_i - k stay continuation cells on row i - k.
    rng = np.random.default_rng([113, every])
    T = 1200
    for _ in range(10):
        p = inputs.draw_params(rng, B)
        _, b, mg = oracle_mod.price(B, p["S0"], p["K"], p["r"], p["q"], p["sigma"], p["expiry"], T,
                                    boundary=True, margin=True, every=every)
        rows = [i for i in range(T - every, -1, -1) if (T - i) % every == 0]
        for i_hi, i_lo in zip(rows, rows[1:]):
            if b[i_hi] < 0 or b[i_hi] == i_hi:
                continue
            if b[i_lo] < b[i_hi] - every:
                assert _near_tie(mg, 2 * i_lo) or _near_tie(mg, 2 * i_lo + 1)
