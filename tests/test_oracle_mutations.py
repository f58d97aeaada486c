"""The pins are strong enough to catch plausible oracle mistakes.

Each case plants one mistake in a private copy of the oracle's C source (on the
CPU, in a temporary directory), builds it, and checks that at least one pin of
``test_oracle_pins`` style rejects it.
"""
import math
import os
import subprocess

import numpy as np
import pytest

from tests import pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "aop_oracle.c")

MUTATIONS = {
    "binomial_weights_swapped": ("const double w_dn = m * (1.0 - p);", "const double w_dn = m * p;"),
    "binomial_exercise_index": ("double e = S * X[2 * j - i + T] - K;\n                int red = (c >= e)",
                                "double e = S * X[2 * j - i + 1 + T] - K;\n                int red = (c >= e)"),
    "binomial_no_dividend_in_p": ("const double p = (exp((r - q) * dt) - d) / (u - d);",
                                  "const double p = (exp(r * dt) - d) / (u - d);"),
    "binomial_tie_goes_green": ("static int is_red(double c, double e)\n{\n    return (c >= e)",
                                "static int is_red(double c, double e)\n{\n    return (c > e)"),
    "trinomial_weights_swapped": ("const double w_d = m * pd, w_o = m * po, w_u = m * pu;",
                                  "const double w_d = m * pu, w_o = m * po, w_u = m * pd;"),
    "trinomial_exercise_index": ("double e = S * X[j - i + T] - K;\n                int red = (c >= e)",
                                 "double e = S * X[j - i + 1 + T] - K;\n                int red = (c >= e)"),
    "trinomial_no_discount": ("const double m = exp(-r * dt);\n    if (!(pu > 0.0",
                              "const double m = 1.0;\n    if (!(pu > 0.0"),
    "bsm_drift_sign": ("const double ca = lam + drift;", "const double ca = lam - drift;"),
    "bsm_drift_sign_b": ("const double cb = lam - drift;", "const double cb = lam + drift;"),
    "bsm_dropped_discount_term": ("const double cc = 1.0 - omega * dtau - 2.0 * lam;",
                                  "const double cc = 1.0 - 2.0 * lam;"),
    "guard_dropped_in_red_test": ("    return (c >= e) && isfinite(c) && isfinite(e);", "    return (c >= e);"),
    "guard_dropped_binomial_loop": ("double e = S * X[2 * j - i + T] - K;\n                int red = (c >= e) & (c < INFINITY) & (e < INFINITY);",
                                    "double e = S * X[2 * j - i + T] - K;\n                int red = (c >= e);"),
    "guard_dropped_trinomial_loop": ("double e = S * X[j - i + T] - K;\n                int red = (c >= e) & (c < INFINITY) & (e < INFINITY);",
                                     "double e = S * X[j - i + T] - K;\n                int red = (c >= e);"),
    "bsm_boundary_off_by_one": ("lastg = green ? k : lastg;", "lastg = green ? k - 1 : lastg;"),
    "bsm_boundary_off_by_one_margin_path": ("                lastg = green ? k : lastg;\n                gap_last", "                lastg = green ? k - 1 : lastg;\n                gap_last"),
    "binomial_boundary_off_by_one": ("last = red ? j : last;\n            }\n        } else {\n            int prev_red = 1;",
                                     "last = red ? j - 1 : last;\n            }\n        } else {\n            int prev_red = 1;"),
    "binomial_boundary_off_by_one_margin_path": ("                last = red ? j : last;\n                gap_last = red ? gap : gap_last;",
                                                 "                last = red ? j - 1 : last;\n                gap_last = red ? gap : gap_last;"),
    "binomial_margin_of_wrong_cell": ("                gap_next = (!red && prev_red) ? -gap : gap_next; /* the cell after a red one */\n                prev_red = red;\n            }\n        }\n        if (boundary) boundary[i] = american ? last : (every == 0 ? -1 : i);\n        if (margin && american) {\n            margin[2 * i] = last >= 0 ? gap_last : NAN;\n            margin[2 * i + 1] = (last + 1 <= i)",
                                      "                gap_next = (!red) ? -gap : gap_next; /* the cell after a red one */\n                prev_red = red;\n            }\n        }\n        if (boundary) boundary[i] = american ? last : (every == 0 ? -1 : i);\n        if (margin && american) {\n            margin[2 * i] = last >= 0 ? gap_last : NAN;\n            margin[2 * i + 1] = (last + 1 <= i)"),
    "bermudan_wrong_exercise_rows": ("(every > 1 && (T - i) % every == 0)", "(every > 1 && (T - i) % every == 1)"),
    "bsm_payoff_shift": ("double g = 1.0 - EX[k + T];\n                int green = g > cont;\n                Vn[k + T] = green ? g : cont;\n                lastg",
                         "double g = 1.0 - EX[k + 1 + T];\n                int green = g > cont;\n                Vn[k + T] = green ? g : cont;\n                lastg"),
}


def _battery(oracle_mod, lib):
    """Return the list of failed pins for one oracle build."""
    fails = []
    P = lambda *a, **k: oracle_mod.price(*a, lib=lib, **k)
    prm = (120.0, 100.0, 0.08, 0.06, 0.3, 1.5)
    try:
        for T in (3, 7):
            for am in (True, False):
                if abs(P(0, *prm, T, american=am) - pins.brute_binomial(*prm, T, american=am)) > 1e-12:
                    fails.append("binomial brute force")
                if abs(P(1, *prm, T, american=am) - pins.brute_trinomial(*prm, T, american=am)) > 1e-12:
                    fails.append("trinomial brute force")
            bp = (90.0, 110.0, 0.08, 0.45, 2.0)
            for am in (True, False):
                got = P(2, bp[0], bp[1], bp[2], 0.0, bp[3], bp[4], T, american=am)
                if abs(got - pins.brute_bsm_put(*bp, T, american=am)) > 1e-12 * bp[1]:
                    fails.append("bsm brute force")
        S, r, q, s, E, T = 120.0, 0.08, 0.01, 0.2, 1.0, 400
        K = 0.5 * S * math.exp(-s * math.sqrt(E * T))
        if abs(P(0, S, K, r, q, s, E, T, american=False) - (S * math.exp(-q * E) - K * math.exp(-r * E))) > 1e-9:
            fails.append("forward identity")
        pr, b, _ = P(0, 100.0, 100.0, 0.05, 0.03, 0.2, 1.0, 200, boundary=True)
        if b[200] != 100:  # S = K, T even: the tie at j = T/2 is red (Definition 2.1)
            fails.append("tie rule")
        if abs(P(2, 100.0, 110.0, 0.05, 0.0, 0.25, 1.0, 1000, american=False) - pins.bs_put(100.0, 110.0, 0.05, 0.25, 1.0)) > 2e-3 * 110:
            fails.append("bsm limit")
        # overflowing lattice tops (sigma sqrt(E T) > 709.8) against high precision
        for model, ref in ((0, pins.mp_binomial), (1, pins.mp_trinomial)):
            ov = (100.0, 100.0, 0.05, 0.03, 80.0, 1.0, 96)
            exact = ref(*ov)
            for kw in ({}, dict(boundary=True, margin=True)):
                got = P(model, *ov, **kw)
                got = got[0] if isinstance(got, tuple) else got
                if not (math.isfinite(got) and abs(got - exact) <= 1e-13 * exact):
                    fails.append("overflow pin")
        # boundaries against decisions recorded on brute-force trees
        none = np.iinfo(np.int64).min
        for T in (6, 8):
            for kw in (dict(boundary=True), dict(boundary=True, margin=True)):
                _, ref = pins.brute_binomial_boundary(*prm, T)
                b = P(0, *prm, T, **kw)[1]
                if any(x != "tie" and int(b[i]) != x for i, x in enumerate(ref)):
                    fails.append("binomial boundary")
                _, ref = pins.brute_bsm_put_boundary(90.0, 110.0, 0.08, 0.45, 2.0, T)
                b = P(2, 90.0, 110.0, 0.08, 0.0, 0.45, 2.0, T, **kw)[1]
                if any(x != "tie" and int(b[i]) != (none if x is None else x) for i, x in enumerate(ref)):
                    fails.append("bsm boundary")
        for T in (6, 9):
            if abs(P(0, *prm, T, every=3) - pins.brute_binomial_bermudan(*prm, T, 3)) > 1e-12:
                fails.append("bermudan brute force")
        # decision gaps at the boundary against a full numpy grid
        gp = (100.0, 95.0, 0.03, 0.05, 0.25, 1.0)
        T = 60
        _, b, mg = P(0, *gp, T, boundary=True, margin=True)
        G, _ = pins.grid_binomial(*gp, T)
        _, u, _, pp, m = pins.bopm_params(*gp[2:], T)
        for i in range(T):
            j = np.arange(i + 1)
            gap = (m * (1 - pp) * G[i + 1, :i + 1] + m * pp * G[i + 1, 1:i + 2] - (gp[0] * u ** (2.0 * j - i) - gp[1])) / gp[1]
            last = int(b[i])
            if 0 <= last and last + 1 <= i and not (abs(mg[2 * i] - gap[last]) <= 1e-12 and
                                                    abs(mg[2 * i + 1] + gap[last + 1]) <= 1e-12):
                fails.append("binomial margins")
                break
    except oracle_mod.OracleError:
        fails.append("rejected a valid option")
    return fails


def test_unmutated_oracle_passes_battery(oracle_mod):
    assert _battery(oracle_mod, None) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(oracle_mod, tmp_path, name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation anchor not found: %s" % name
    mutated = src.replace(old, new, 1)
    c = tmp_path / "m.c"
    c.write_text(mutated)
    so = tmp_path / "m.so"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(so), str(c), "-lm"],
                   check=True)
    lib = oracle_mod.load_variant(str(so))
    assert _battery(oracle_mod, lib), "planted mistake %s was not caught" % name
