"""CPU model of the GPU solver's schedule (test double, not product code).

Mirrors the control flow of ``aop_solver.hip`` step for step -- the same
trapezoid frames, band walkers with their ballot/clamp rule, middle-row arena,
FFT correlation with the closed-form kernel spectrum -- in numpy, with every
buffer access bounds-checked.  It lets the CPU suite exercise every geometry
(all-red rows, all-green shortcut, clamped heights, odd heights, the BSM cone
edges) and record the recursion's depth and arena use, without a GPU.
"""
from __future__ import annotations

import math

import numpy as np

BAND = 128       # BSM band walker: two cells per lane
BAND_LAT = 128   # lattice band walker: two cells per lane
BINOMIAL, TRINOMIAL, BSM = 0, 1, 2
NONE = np.iinfo(np.int64).min


class Geometry(Exception):
    pass


class Buf:
    """A double buffer addressed by absolute index, with bounds checks."""

    def __init__(self, lo: int, hi: int, name: str):
        self.lo, self.hi, self.name = lo, hi, name
        self.a = np.full(hi - lo + 1, np.nan)

    def _chk(self, i0, i1):
        if i1 < i0:
            return
        if i0 < self.lo or i1 > self.hi:
            raise Geometry("%s access [%d,%d] outside [%d,%d]" % (self.name, i0, i1, self.lo, self.hi))

    def get(self, i0, i1):
        self._chk(i0, i1)
        return self.a[i0 - self.lo:i1 - self.lo + 1].copy()

    def put(self, i0, vals):
        vals = np.asarray(vals, dtype=float)
        self._chk(i0, i0 + len(vals) - 1)
        self.a[i0 - self.lo:i0 - self.lo + len(vals)] = vals


def params(opt, lam=1.0 / 3.0):
    m_, T = opt["model"], opt["T"]
    S, K, r, q, sig, E = opt["S0"], opt["K"], opt["r"], opt["q"], opt["sigma"], opt["expiry"]
    d = dict(model=m_, T=T, S=S, K=K, s0=0.0)
    if m_ == BINOMIAL:
        dt = E / T
        a = sig * math.sqrt(dt)
        u = math.exp(a)
        dn = 1 / u
        p = (math.exp((r - q) * dt) - dn) / (u - dn)
        m = math.exp(-r * dt)
        d.update(a=a, w=(m * (1 - p), m * p, 0.0))
    elif m_ == TRINOMIAL:
        dt = E / T
        A = sig * math.sqrt(2 * dt)
        su, sd = math.exp(A / 2), math.exp(-A / 2)
        g = math.exp((r - q) * dt / 2)
        pu = ((g - sd) / (su - sd)) ** 2
        pd = ((su - g) / (su - sd)) ** 2
        po = 1 - pu - pd
        m = math.exp(-r * dt)
        d.update(a=A, w=(m * pd, m * po, m * pu))
    else:
        dtau = 0.5 * sig * sig * E / T
        ds = math.sqrt(dtau / lam)
        om = 2 * r / sig ** 2
        la = dtau / ds ** 2
        dr = 0.5 * (om - 1) * dtau / ds
        d.update(a=ds, s0=math.log(S / K), w=(la - dr, 1 - om * dtau - 2 * la, la + dr))
    return d


def ex_bin(d, i, j):
    return d["S"] * np.exp(np.asarray(2 * j - i, dtype=float) * d["a"]) - d["K"]


def ex_tri(d, i, j):
    return d["S"] * np.exp(np.asarray(j - i, dtype=float) * d["a"]) - d["K"]


def ex_bsm(d, k):
    return 1.0 - np.exp(d["s0"] + np.asarray(k, dtype=float) * d["a"])


def red_of(c, e):
    with np.errstate(invalid="ignore"):
        return (c >= e) & (c < np.inf) & (e < np.inf)


def kernel_power(d, h, N, beta=0.0, lscale=0.0):
    f = np.arange(N)
    ff = np.where(f <= N // 2, f, f - N)
    x = ff / N
    s = np.sin(np.pi * x) ** 2
    sn, cs = np.sin(2 * np.pi * x), np.cos(2 * np.pi * x)
    if d["model"] == BINOMIAL:
        wd, wu = d["w"][0], d["w"][1] * math.exp(beta)
        rho = wd + wu
        lg = np.log1p(-4 * wd * wu * s / rho ** 2)
        arg = np.arctan2(wu * sn, wd + wu * cs)
    else:
        wm, wc, wp = d["w"]
        wm, wp = wm * math.exp(-beta), wp * math.exp(beta)
        rho = wm + wc + wp
        sp, df = wp + wm, wp - wm
        delta = (-4 * s * (rho * sp - df * df) + 16 * wp * wm * s * s) / rho ** 2
        with np.errstate(divide="ignore"):
            lg = np.log1p(delta)
        arg = np.arctan2(df * sn, rho - 2 * sp * s)
    lrel = 0.5 * h * lg
    mag = np.where(lrel > -60, np.exp(h * math.log(rho) + np.maximum(lrel, -700) + lscale), 0.0)
    return mag * np.exp(1j * h * arg)


class Model:
    def __init__(self, opt, lam=1.0 / 3.0):
        self.d = params(opt, lam)
        self.T = opt["T"]
        self.no_green = opt["model"] != BSM and opt["q"] == 0.0 and opt["r"] >= 0.0
        self.bnd = np.full(self.T + 1, -7, dtype=np.int64)
        self.max_depth = 0
        self.ffts = []  # (N, h)
        self.band_rows = 0

    # FFT correlation: dst[t] = (x * W^h)[out_off + t]
    def correlate(self, src: Buf, s0, n_in, h, out_off, n_out, dst: Buf, d0, beta=0.0, tc=0.0):
        if n_out <= 0:
            return
        x = src.get(s0, s0 + n_in - 1)
        if beta != 0.0:
            t = np.arange(n_in)
            nz = x != 0
            x = np.where(nz, x * np.exp(np.where(nz, -beta * (t - tc), 0.0)), 0.0)
        if np.isnan(x).any():
            raise Geometry("correlate reads unset cells")
        N = 1 << max(1, math.ceil(math.log2(n_in)))
        if out_off + n_out > n_in:
            raise Geometry("window wraps")
        X = np.fft.fft(x, N)
        y = np.fft.ifft(X * kernel_power(self.d, h, N, beta, -beta * tc)).real
        self.ffts.append((N, h))
        m = np.arange(out_off, out_off + n_out)
        dst.put(d0, y[out_off:out_off + n_out] * (np.exp(beta * m) if beta != 0.0 else 1.0))

    # ----------------------------------------------------------- bands
    def band_lat(self, i0, c0, h, b, src: Buf, dst: Buf):
        d, tri = self.d, self.d["model"] == TRINOMIAL
        ex = ex_tri if tri else ex_bin
        wmax = (lambda i: 2 * i) if tri else (lambda i: i)
        if b - c0 + 1 > BAND_LAT:
            raise Geometry("band too narrow")
        j = c0 + np.arange(BAND_LAT)
        g = np.where(j <= wmax(i0), ex(d, i0, j), 0.0)
        if b >= c0:
            g[:b - c0 + 1] = src.get(c0, b)
        bc = b
        for k in range(1, h + 1):
            i = i0 - k
            gn1 = np.append(g[1:], ex(d, i + 1, c0 + BAND_LAT))
            if tri:
                gn2 = np.append(g[2:], [ex(d, i + 1, c0 + BAND_LAT), ex(d, i + 1, c0 + BAND_LAT + 1)])
                c = d["w"][0] * g + d["w"][1] * gn1 + d["w"][2] * gn2
            else:
                c = d["w"][0] * g + d["w"][1] * gn1
            e = ex(d, i, j)
            red = c >= e
            g = np.maximum(c, e)
            if tri and bc >= 2 * (i + 1):  # previous row entirely red
                rr = red & (j <= wmax(i))
                bc = max(c0 + int(np.nonzero(rr)[0].max()) if rr.any() else c0 - 1, c0 - 1)
            elif bc >= c0:  # the previous boundary cell stays red, or the boundary drops by one
                if bc > wmax(i) or not red[bc - c0]:
                    bc -= 1
            self.bnd[i] = bc
            self.band_rows += 1
        if bc >= c0:
            dst.put(c0, g[:bc - c0 + 1])
        return bc, g[0]

    def band_bsm(self, n0, f, h, R0, src: Buf, dst: Buf):
        d, T = self.d, self.T
        base = R0 - (BAND - 1)
        k = base + np.arange(BAND)
        v = ex_bsm(d, k)
        if R0 >= f + 1:
            v[f + 1 - base:] = src.get(f + 1, R0)
        fc = f
        wm, wc, wp = d["w"]
        for t in range(1, h + 1):
            base -= 1
            k = base + np.arange(BAND)
            vm2 = np.concatenate([[ex_bsm(d, k[0] - 1), ex_bsm(d, k[0])], v[:-2]])
            vm1 = np.concatenate([[ex_bsm(d, k[0])], v[:-1]])
            cont = wm * vm2 + wc * vm1 + wp * v
            g = ex_bsm(d, k)
            green = g > cont
            v = np.maximum(cont, g)
            lf = fc - base
            if 0 <= lf < BAND and not green[lf]:
                fc -= 1
            n = n0 + t
            self.bnd[n] = NONE if fc < -(T - n) else min(fc, T - n)
            self.band_rows += 1
        sel = (k > fc) & (k <= R0 - h)
        if sel.any():
            ks = k[sel]
            dst.put(int(ks[0]), v[sel])
        return fc, v[-1]

    # ------------------------------------------------------ recursion
    def solve_lat(self, i0, c0, h, b, src: Buf, dst: Buf, depth=0):
        self.max_depth = max(self.max_depth, depth)
        span = 2 if self.d["model"] == TRINOMIAL else 1
        nred = b - c0 + 1
        if nred <= BAND_LAT:
            return self.band_lat(i0, c0, h, b, src, dst)[0]
        h1, h2 = h // 2, h - h // 2
        mid = Buf(c0, b, "mid")
        self.correlate(src, c0, nred, h1, 0 if span == 1 else h1, nred - span * h1, mid, c0)
        br = self.solve_lat(i0, b - span * h1 + 1, h1, b, src, mid, depth + 1)
        n2 = br - c0 + 1
        if n2 - span * h2 > 0:
            self.correlate(mid, c0, n2, h2, 0 if span == 1 else h2, n2 - span * h2, dst, c0)
        return self.solve_lat(i0 - h1, br - span * h2 + 1, h2, br, mid, dst, depth + 1)

    def solve_bsm(self, n, f, h, src: Buf, dst: Buf, depth=0):
        self.max_depth = max(self.max_depth, depth)
        if h <= (BAND - 2) // 2:
            return self.band_bsm(n, f, h, f + 2 * h, src, dst)[0]
        h1, h2 = h // 2, h - h // 2
        mid = Buf(f - h1 + 1, f + h + h2, "mid")
        self.correlate(src, f + 1, 2 * h, h1, h1, 2 * h - 2 * h1, mid, f + 1 + h1)
        fp = self.solve_bsm(n, f, h1, src, mid, depth + 1)
        if not (f - h1 <= fp <= f):
            raise Geometry("bsm boundary left its range")
        nin = f + h + h2 - fp
        self.correlate(mid, fp + 1, nin, h2, h2, nin - 2 * h2, dst, fp + 1 + h2)
        return self.solve_bsm(n + h1, fp, h2, mid, dst, depth + 1)

    # ---------------------------------------------------------- drivers
    def price(self):
        return self._bsm() if self.d["model"] == BSM else self._lattice()

    def _lattice(self):
        d, T = self.d, self.T
        tri = d["model"] == TRINOMIAL
        ex = ex_tri if tri else ex_bin
        wT = 2 * T if tri else T
        A = Buf(0, wT + 2, "rowA")
        B = Buf(0, wT + 2, "rowB")
        j = np.arange(wT + 1)
        eT = ex(d, T, j)
        rT = red_of(0.0, eT)
        gT = np.where(rT, 0.0, eT)
        self.bnd[T] = int(j[rT].max()) if rT.any() else -1
        w1 = wT - (2 if tri else 1)
        jj = np.arange(w1 + 1)
        if tri:
            c = d["w"][0] * gT[:w1 + 1] + d["w"][1] * gT[1:w1 + 2] + d["w"][2] * gT[2:w1 + 3]
        else:
            c = d["w"][0] * gT[:w1 + 1] + d["w"][1] * gT[1:w1 + 2]
        e = ex(d, T - 1, jj)
        red = red_of(c, e)
        A.put(0, np.where(red, c, e))
        b = int(jj[red].max()) if red.any() else -1
        self.bnd[T - 1] = b
        i0, src, dst = T - 1, A, B
        if T > 1 and (b == w1 or self.no_green):
            b = w1
            self.bnd[T - 1] = b
            # all-red row T-1: one tilted correlation to the root
            beta = d["a"] * (1.0 if tri else 2.0)
            tc = (T - 1) + math.log(d["K"] / d["S"]) / d["a"] if tri else 0.5 * ((T - 1) + math.log(d["K"] / d["S"]) / d["a"])
            tc = min(max(tc, 0.0), float(b))
            self.bnd[:T - 1] = [2 * i if tri else i for i in range(T - 1)]
            out = Buf(0, 0, "val")
            hh = T - 1
            self.correlate(src, 0, b + 1, hh, hh if tri else 0, 1, out, 0, beta, tc)
            return out.get(0, 0)[0]
        while i0 > 0:
            if b < 0:
                self.bnd[:i0] = -1
                return d["S"] - d["K"]
            nred = b + 1
            if nred <= BAND_LAT:
                _, v0 = self.band_lat(i0, 0, i0, b, src, dst)
                return v0
            h = nred if not tri else nred // 2
            h = min(h, i0)
            b = self.solve_lat(i0, 0, h, b, src, dst)
            i0 -= h
            src, dst = dst, src
        return src.get(0, 0)[0] if b >= 0 else d["S"] - d["K"]

    def _bsm(self):
        d, T = self.d, self.T
        A = Buf(-2 * T - 1, T + 1, "rowA")
        B = Buf(-2 * T - 1, T + 1, "rowB")
        k = np.arange(-T, T + 1)
        g = ex_bsm(d, k)
        self.bnd[0] = int(k[g > 0].max()) if (g > 0).any() else NONE
        v0 = np.maximum(g, 0.0)
        kk = k[1:-1]
        cont = d["w"][0] * v0[:-2] + d["w"][1] * v0[1:-1] + d["w"][2] * v0[2:]
        g1 = g[1:-1]
        green = g1 > cont
        if len(kk):
            A.put(int(kk[0]), np.where(green, g1, cont))
        f1 = int(kk[green].max()) if green.any() else NONE
        self.bnd[1] = f1
        n, R, L = 1, T - 1, -(T - 1)
        f = L - 1 if f1 == NONE else f1
        src, dst = A, B
        while True:
            if n == T:
                return d["K"] * (ex_bsm(d, 0) if f >= 0 else src.get(0, 0)[0])
            if f < L:
                for m in range(n + 1, T + 1):
                    self.bnd[m] = NONE
                out = Buf(0, 0, "val")
                hh = T - n
                self.correlate(src, L, R - L + 1, hh, hh, 1, out, 0)
                return d["K"] * out.get(0, 0)[0]
            if f >= R:
                for m in range(n + 1, T + 1):
                    self.bnd[m] = T - m
                return d["K"] * ex_bsm(d, 0)
            w = R - f
            if w <= BAND - 2:
                _, vr = self.band_bsm(n, f, T - n, R, src, dst)
                return d["K"] * vr
            h = min(w // 2, T - n)
            fn = self.solve_bsm(n, f, h, src, dst)
            self.correlate(src, f + 1, w, h, h, w - 2 * h, dst, f + 1 + h)
            n, R, L, f = n + h, R - h, L + h, fn
            src, dst = dst, src
