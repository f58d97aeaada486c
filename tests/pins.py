"""Independent references that pin the oracle (test code, not product code).

Each function restates a fact the paper's formulas fix, in a form that does not
share structure with the oracle's in-place backward induction:

* brute-force non-recombining trees / grids (every path enumerated, node
  prices carried along the path) -- Fig. 1 and Definition 2.1 (binomial),
  Sec. 3 (trinomial), eq. (bsmG) (BSM);
* closed-form European lattice sums (binomial distribution in log space,
  multinomial expansion of the BSM scheme);
* the Black-Scholes(-Merton) closed forms the lattices converge to;
* a high-precision (mpmath) evaluation of the binomial lattice.
"""
from __future__ import annotations

import math

import mpmath


# ----------------------------------------------------------------- parameters
def bopm_params(r, q, sigma, E, T):
    """CRR parameters of Fig. 1: dt, u, d, p, m."""
    dt = E / T
    u = math.exp(sigma * math.sqrt(dt))
    d = 1.0 / u
    p = (math.exp((r - q) * dt) - d) / (u - d)
    m = math.exp(-r * dt)
    return dt, u, d, p, m


def topm_params(r, q, sigma, E, T):
    """Trinomial parameters of Sec. 3: u = e^{V sqrt(2 dt)}, p_u, p_d, p_o."""
    dt = E / T
    u = math.exp(sigma * math.sqrt(2.0 * dt))
    su, sd = math.sqrt(u), math.sqrt(1.0 / u)
    g = math.exp((r - q) * dt / 2.0)
    pu = ((g - sd) / (su - sd)) ** 2
    pd = ((su - g) / (su - sd)) ** 2
    po = 1.0 - pu - pd
    m = math.exp(-r * dt)
    return dt, u, pu, po, pd, m


def bsm_coeffs(r, sigma, E, T, lam=1.0 / 3.0):
    """eq. (bsmG) coefficients: a on v_{k+1}, b on v_{k-1}, c on v_k; ds, dtau."""
    dtau = 0.5 * sigma * sigma * E / T
    ds = math.sqrt(dtau / lam)
    omega = 2.0 * r / (sigma * sigma)
    a = dtau / ds ** 2 + (omega - 1.0) / 2.0 * dtau / ds
    b = dtau / ds ** 2 - (omega - 1.0) / 2.0 * dtau / ds
    c = 1.0 - omega * dtau - 2.0 * dtau / ds ** 2
    return a, b, c, ds, dtau


# -------------------------------------------------------------- brute force
def brute_binomial(S, K, r, q, sigma, E, T, american=True):
    """Non-recombining binomial tree: 2^T paths, price carried along each path."""
    _, u, d, p, m = bopm_params(r, q, sigma, E, T)

    def value(t, x):
        ex = x - K
        if t == T:
            return max(ex, 0.0)
        cont = m * (p * value(t + 1, x * u) + (1.0 - p) * value(t + 1, x * d))
        return max(cont, ex) if american else cont

    return value(0, S)


def brute_trinomial(S, K, r, q, sigma, E, T, american=True):
    """Non-recombining trinomial tree: 3^T paths."""
    _, u, pu, po, pd, m = topm_params(r, q, sigma, E, T)

    def value(t, x):
        ex = x - K
        if t == T:
            return max(ex, 0.0)
        cont = m * (pu * value(t + 1, x * u) + po * value(t + 1, x) + pd * value(t + 1, x / u))
        return max(cont, ex) if american else cont

    return value(0, S)


def brute_bsm_put(S, K, r, sigma, E, T, american=True, lam=1.0 / 3.0):
    """Explicit scheme evaluated path by path from the apex: 3^T paths."""
    a, b, c, ds, _ = bsm_coeffs(r, sigma, E, T, lam)

    def value(n, s):  # n = steps of time to expiry left
        g = 1.0 - math.exp(s)
        if n == 0:
            return max(g, 0.0)
        cont = b * value(n - 1, s - ds) + c * value(n - 1, s) + a * value(n - 1, s + ds)
        return max(cont, g) if american else cont

    return K * value(T, math.log(S / K))


# --------------------------------------------------------- closed-form sums
def european_binomial_sum(S, K, r, q, sigma, E, T):
    """sum_k C(T,k) p^k (1-p)^(T-k) m^T (S u^(2k-T) - K)^+ in log space."""
    _, u, _, p, m = bopm_params(r, q, sigma, E, T)
    lu, lp, lq, lm = math.log(u), math.log(p), math.log1p(-p), math.log(m)
    lgT = math.lgamma(T + 1)
    tot = 0.0
    for k in range(T + 1):
        x = S * math.exp((2 * k - T) * lu)
        if x <= K:
            continue
        lw = lgT - math.lgamma(k + 1) - math.lgamma(T - k + 1) + k * lp + (T - k) * lq + T * lm
        tot += math.exp(lw) * (x - K)
    return tot


def european_bsm_multinomial(S, K, r, sigma, E, T, lam=1.0 / 3.0):
    """Apex value of the linear scheme as a multinomial sum over step counts.

    A path of T steps with n_a moves to k+1 (weight a), n_b to k-1 (weight b)
    and the rest staying (weight c) ends at k = n_a - n_b.
    """
    a, b, c, ds, _ = bsm_coeffs(r, sigma, E, T, lam)
    s0 = math.log(S / K)
    la, lb = math.log(a), math.log(b)
    lc = math.log(c) if c > 0 else -math.inf
    lgT = math.lgamma(T + 1)
    tot = 0.0
    for na in range(T + 1):
        for nb in range(T + 1 - na):
            nc = T - na - nb
            if nc > 0 and c == 0:
                continue
            pay = 1.0 - math.exp(s0 + (na - nb) * ds)
            if pay <= 0:
                continue
            lw = lgT - math.lgamma(na + 1) - math.lgamma(nb + 1) - math.lgamma(nc + 1) + na * la + nb * lb
            if nc:
                lw += nc * lc
            tot += math.exp(lw) * pay
    return K * tot


def bs_call_div(S, K, r, q, sigma, E):
    """Black-Scholes-Merton European call with continuous dividend yield."""
    d1 = (math.log(S / K) + (r - q + 0.5 * sigma * sigma) * E) / (sigma * math.sqrt(E))
    d2 = d1 - sigma * math.sqrt(E)
    N = lambda x: 0.5 * math.erfc(-x / math.sqrt(2.0))
    return S * math.exp(-q * E) * N(d1) - K * math.exp(-r * E) * N(d2)


def bs_put(S, K, r, sigma, E):
    d1 = (math.log(S / K) + (r + 0.5 * sigma * sigma) * E) / (sigma * math.sqrt(E))
    d2 = d1 - sigma * math.sqrt(E)
    N = lambda x: 0.5 * math.erfc(-x / math.sqrt(2.0))
    return K * math.exp(-r * E) * N(-d2) - S * N(-d1)


# --------------------------------------------------------- high precision
def mp_binomial(S, K, r, q, sigma, E, T, american=True, dps=50):
    """Binomial lattice of Definition 2.1 evaluated in mpmath at ``dps`` digits."""
    with mpmath.workdps(dps):
        S, K, r, q, sigma, E = (mpmath.mpf(x) for x in (S, K, r, q, sigma, E))
        dt = E / T
        u = mpmath.e ** (sigma * mpmath.sqrt(dt))
        d = 1 / u
        p = (mpmath.e ** ((r - q) * dt) - d) / (u - d)
        m = mpmath.e ** (-r * dt)
        row = [max(S * u ** (2 * j - T) - K, 0) for j in range(T + 1)]
        for i in range(T - 1, -1, -1):
            new = []
            for j in range(i + 1):
                c = m * ((1 - p) * row[j] + p * row[j + 1])
                new.append(max(c, S * u ** (2 * j - i) - K) if american else c)
            row = new
        return float(row[0])


# ---------------------------------------------------------- numpy full grid
def grid_binomial(S, K, r, q, sigma, E, T):
    """Full (T+1)x(T+1) grid and red mask of Definition 2.1, row by row (numpy)."""
    import numpy as np

    _, u, _, p, m = bopm_params(r, q, sigma, E, T)
    G = np.full((T + 1, T + 1), np.nan)
    red = np.zeros((T + 1, T + 1), dtype=bool)
    j = np.arange(T + 1)
    e = S * u ** (2.0 * j - T) - K
    G[T] = np.maximum(e, 0.0)
    red[T] = 0.0 >= e
    for i in range(T - 1, -1, -1):
        j = np.arange(i + 1)
        c = m * (1 - p) * G[i + 1, :i + 1] + m * p * G[i + 1, 1:i + 2]
        e = S * u ** (2.0 * j - i) - K
        red[i, :i + 1] = c >= e
        G[i, :i + 1] = np.where(c >= e, c, e)
    return G, red


def mp_trinomial(S, K, r, q, sigma, E, T, american=True, dps=50):
    """Trinomial lattice of Sec. 3 evaluated in mpmath at ``dps`` digits."""
    with mpmath.workdps(dps):
        S, K, r, q, sigma, E = (mpmath.mpf(x) for x in (S, K, r, q, sigma, E))
        dt = E / T
        A = sigma * mpmath.sqrt(2 * dt)
        su, sd = mpmath.e ** (A / 2), mpmath.e ** (-A / 2)
        g = mpmath.e ** ((r - q) * dt / 2)
        pu = ((g - sd) / (su - sd)) ** 2
        pd = ((su - g) / (su - sd)) ** 2
        po = 1 - pu - pd
        m = mpmath.e ** (-r * dt)
        u = mpmath.e ** A
        row = [max(S * u ** (j - T) - K, 0) for j in range(2 * T + 1)]
        for i in range(T - 1, -1, -1):
            new = []
            for j in range(2 * i + 1):
                c = m * (pd * row[j] + po * row[j + 1] + pu * row[j + 2])
                new.append(max(c, S * u ** (j - i) - K) if american else c)
            row = new
        return float(row[0])


def grid_trinomial(S, K, r, q, sigma, E, T):
    """Full trinomial grid (row i: columns 0..2i) and red mask, row by row (numpy)."""
    import numpy as np

    _, u, pu, po, pd, m = topm_params(r, q, sigma, E, T)
    G = np.full((T + 1, 2 * T + 1), np.nan)
    red = np.zeros((T + 1, 2 * T + 1), dtype=bool)
    j = np.arange(2 * T + 1)
    e = S * u ** (j - float(T)) - K
    G[T] = np.maximum(e, 0.0)
    red[T] = 0.0 >= e
    for i in range(T - 1, -1, -1):
        w = 2 * i + 1
        j = np.arange(w)
        c = m * pd * G[i + 1, :w] + m * po * G[i + 1, 1:w + 1] + m * pu * G[i + 1, 2:w + 2]
        e = S * u ** (j - float(i)) - K
        red[i, :w] = c >= e
        G[i, :w] = np.where(c >= e, c, e)
    return G, red


def grid_bsm_put(S, K, r, sigma, E, T, lam=1.0 / 3.0):
    """Full explicit BSM grid on the apex's cone and its exercise mask (numpy).

    Row n (n = 0 at expiry, T at the apex) holds offsets k = -T..T at column
    k + T; only |k| <= T - n is defined.  Returns (V, green) with green[n, k+T]
    true where the exercise value exceeds the continuation value.
    """
    import numpy as np

    a, b, c, ds, _ = bsm_coeffs(r, sigma, E, T, lam)
    s0 = math.log(S / K)
    k = np.arange(-T, T + 1)
    g = 1.0 - np.exp(s0 + k * ds)
    V = np.full((T + 1, 2 * T + 1), np.nan)
    green = np.zeros((T + 1, 2 * T + 1), dtype=bool)
    V[0] = np.maximum(g, 0.0)
    green[0] = g > 0.0
    for n in range(1, T + 1):
        lo, hi = n, 2 * T - n  # columns of |k| <= T - n
        cont = b * V[n - 1, lo - 1:hi] + c * V[n - 1, lo:hi + 1] + a * V[n - 1, lo + 1:hi + 2]
        gg = g[lo:hi + 1]
        green[n, lo:hi + 1] = gg > cont
        V[n, lo:hi + 1] = np.where(gg > cont, gg, cont)
    return V, green


# ----------------------------------------- brute-force exercise decisions
def _decisions_to_boundary(red_at, green_at, T, width, lattice=True):
    """Per-row boundary from node decisions recorded along every tree path.

    Lattices: last red column of each row (-1 if none).  BSM: last green
    offset (None if none).  A row whose decisions disagree between paths (a
    rounding-level tie reached by differently rounded products) is None.
    """
    out = []
    for t in range(T + 1):
        cols = range(width(t))
        amb = any((t, j) in red_at and (t, j) in green_at for j in cols)
        if amb:
            out.append("tie")
            continue
        if lattice:
            reds = [j for j in cols if (t, j) in red_at]
            out.append(max(reds) if reds else -1)
        else:
            greens = [j for j in cols if (t, j) in green_at]
            out.append(max(greens) if greens else None)
    return out


def brute_binomial_boundary(S, K, r, q, sigma, E, T):
    """Boundary of each row from a non-recombining tree walked path by path.

    Node (t, j) is reached after j up moves; its price is carried along the
    path by multiplying with u or d.  Returns (price, boundary list)."""
    _, u, d, p, m = bopm_params(r, q, sigma, E, T)
    red_at, green_at = set(), set()

    def value(t, j, x):
        ex = x - K
        if t == T:
            (red_at if 0.0 >= ex else green_at).add((t, j))
            return max(ex, 0.0)
        cont = m * (p * value(t + 1, j + 1, x * u) + (1.0 - p) * value(t + 1, j, x * d))
        (red_at if cont >= ex else green_at).add((t, j))
        return max(cont, ex)

    price = value(0, 0, S)
    return price, _decisions_to_boundary(red_at, green_at, T, lambda t: t + 1)


def brute_trinomial_boundary(S, K, r, q, sigma, E, T):
    """As brute_binomial_boundary for the trinomial tree (children j, j+1, j+2)."""
    _, u, pu, po, pd, m = topm_params(r, q, sigma, E, T)
    red_at, green_at = set(), set()

    def value(t, j, x):
        ex = x - K
        if t == T:
            (red_at if 0.0 >= ex else green_at).add((t, j))
            return max(ex, 0.0)
        cont = m * (pu * value(t + 1, j + 2, x * u) + po * value(t + 1, j + 1, x) + pd * value(t + 1, j, x / u))
        (red_at if cont >= ex else green_at).add((t, j))
        return max(cont, ex)

    price = value(0, 0, S)
    return price, _decisions_to_boundary(red_at, green_at, T, lambda t: 2 * t + 1)


def brute_bsm_put_boundary(S, K, r, sigma, E, T, lam=1.0 / 3.0):
    """Exercise decisions of the explicit scheme walked path by path from the apex.

    Returns (price, boundary) with boundary[n] the last exercise offset k of
    step n (n = 0 at expiry), None if none, "tie" if paths disagree."""
    a, b, c, ds, _ = bsm_coeffs(r, sigma, E, T, lam)
    red_at, green_at = set(), set()

    def value(n, k, s):  # n = steps to expiry left, k = offset from the apex
        g = 1.0 - math.exp(s)
        if n == 0:
            (green_at if g > 0.0 else red_at).add((n, k + T))
            return max(g, 0.0)
        cont = b * value(n - 1, k - 1, s - ds) + c * value(n - 1, k, s) + a * value(n - 1, k + 1, s + ds)
        (green_at if g > cont else red_at).add((n, k + T))
        return max(cont, g)

    price = K * value(T, 0, math.log(S / K))
    bnd = _decisions_to_boundary(red_at, green_at, T, lambda n: 2 * T + 1, lattice=False)
    return price, [x - T if isinstance(x, int) else x for x in bnd]


def brute_binomial_bermudan(S, K, r, q, sigma, E, T, every):
    """Non-recombining binomial tree with exercise only at depths t (time
    steps from today) where (T - t) % every == 0, t < T (and the payoff at T)."""
    _, u, d, p, m = bopm_params(r, q, sigma, E, T)

    def value(t, x):
        ex = x - K
        if t == T:
            return max(ex, 0.0)
        cont = m * (p * value(t + 1, x * u) + (1.0 - p) * value(t + 1, x * d))
        return max(cont, ex) if (T - t) % every == 0 else cont

    return value(0, S)
