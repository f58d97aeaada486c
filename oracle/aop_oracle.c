/*
 * aop_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct CPU reference for American option pricing on
 * the three lattices/grids of Ahmad et al., "Fast American Option Pricing using
 * Nonlinear Stencils" (arXiv 2303.02317).  It is the Theta(T^2) backward
 * induction over the full lattice or grid, in IEEE double precision, with no
 * blocking, fusion or reordering beyond the definitions:
 *
 *   binomial call   -- Fig. 1 (standard looping code) and Definition 2.1 of
 *                      Sec. 2: G[i][j] = max(s0*G[i+1][j] + s1*G[i+1][j+1],
 *                      S*u^(2j-i) - K), down child weighted m(1-p), up child mp.
 *   trinomial call  -- Sec. 3 / appendix Sec. A.1: children j, j+1, j+2 with
 *                      weights m*p_d, m*p_o, m*p_u, exercise S*u^(j-i) - K,
 *                      row i holding columns 0..2i.
 *   BSM put         -- Sec. 4.2, eq. (bsmG): explicit finite differences for the
 *                      nondimensional Black-Scholes-Merton complementarity
 *                      problem in s = ln(x/K), tau = sigma^2 (E - t) / 2.
 *
 * Nothing in the GPU library includes, links or calls this file, and this file
 * includes nothing from it.  Only tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes): E is in years and dt = E/T; ties go to the continuation ("red")
 * value, as in Definition 2.1; a cell whose exercise or continuation value is
 * not finite is an exercise ("green") cell, so that overflowed deep
 * in-the-money cells cannot pose as continuation cells; the BSM grid is
 * centred on s0 = ln(S0/K), uses lambda = dtau/ds^2 with dtau = sigma^2 E /
 * (2T), and prices on the dependency cone of the apex (2T+1 points at expiry).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL 1
#define OR_EPROB 2
#define OR_ENOMEM 3

#define OR_BINOMIAL 0
#define OR_TRINOMIAL 1
#define OR_BSM_PUT 2


/* Red ("continuation") decision of Definition 2.1: ties go to red; a non-finite
 * value marks the exercise side (deep in the money, overflowed). */
static int is_red(double c, double e)
{
    return (c >= e) && isfinite(c) && isfinite(e);
}

/*
 * Binomial (CRR) American or European call -- Fig. 1, Definition 2.1.
 * boundary[i] = last red column of row i (or -1), i = 0..T.
 * margin[2i]   = (c-e)/K at the last red cell of row i (NAN if none),
 * margin[2i+1] = (e-c)/K at the cell right after it (NAN if none).
 * Below row T the two gaps are kept as the row is swept (the gap of the last
 * red cell seen so far and of the cell right after it), so recording them
 * costs no extra array traffic.
 * (Margins are decision gaps in units of the strike; -inf marks non-finite.)
 */
static int oracle_binomial(double S, double K, double r, double q, double sigma, double E,
                           int64_t T, int64_t every, double *price, int64_t *boundary,
                           double *margin)
{
    const double dt = E / (double)T;
    const double a = sigma * sqrt(dt);
    const double u = exp(a);
    const double d = 1.0 / u;
    const double p = (exp((r - q) * dt) - d) / (u - d);
    const double m = exp(-r * dt);
    if (!(p > 0.0 && p < 1.0))
        return OR_EPROB;
    const double w_dn = m * (1.0 - p); /* weight on G[i+1][j]   (down move) */
    const double w_up = m * p;         /* weight on G[i+1][j+1] (up move)   */

    double *X = (double *)malloc(sizeof(double) * (size_t)(2 * T + 1)); /* X[k+T] = e^{k a} */
    double *G = (double *)malloc(sizeof(double) * (size_t)(T + 1));
    double *D = margin ? (double *)malloc(sizeof(double) * (size_t)(T + 1)) : NULL;
    if (!X || !G || (margin && !D)) {
        free(X); free(G); free(D);
        return OR_ENOMEM;
    }
    for (int64_t k = -T; k <= T; ++k)
        X[k + T] = exp((double)k * a);

    /* Expiry row T: G^red = 0, G^green = S u^{2j-T} - K. */
    int64_t last = -1;
    for (int64_t j = 0; j <= T; ++j) {
        double e = S * X[2 * j - T + T] - K;
        int red = is_red(0.0, e);
        G[j] = red ? 0.0 : e;
        if (D) D[j] = 0.0 - e;
        if (red) last = j;
    }
    if (boundary) boundary[T] = last;
    if (margin) {
        margin[2 * T] = last >= 0 ? D[last] / K : NAN;
        margin[2 * T + 1] = (last + 1 <= T) ? -D[last + 1] / K : NAN;
    }

    /* Rows T-1 .. 0, in place: G[j] <- f(G[j], G[j+1]).  The three loop
     * bodies are the same recurrence; they differ only in what they record.
     * every: 1 American (exercise on every row), 0 European (never before
     * expiry), d >= 2 Bermudan: exercise on the rows i with (T - i) % d == 0,
     * every d steps back from expiry; on the other rows every cell is a
     * continuation (red) cell. */
    double gap_last = NAN, gap_next = NAN; /* decision gaps at the last red cell and the next */
    for (int64_t i = T - 1; i >= 0; --i) {
        last = -1;
        const int american = every == 1 || (every > 1 && (T - i) % every == 0);
        if (!american) {
            for (int64_t j = 0; j <= i; ++j)
                G[j] = w_dn * G[j] + w_up * G[j + 1];
        } else if (!D) {
            for (int64_t j = 0; j <= i; ++j) {
                double c = w_dn * G[j] + w_up * G[j + 1];
                double e = S * X[2 * j - i + T] - K;
                int red = (c >= e) & (c < INFINITY) & (e < INFINITY); /* is_red() */
                G[j] = red ? c : e;
                last = red ? j : last;
            }
        } else {
            int prev_red = 1; /* column -1 counts as red: with no red cell the next cell is column 0 */
            for (int64_t j = 0; j <= i; ++j) {
                double c = w_dn * G[j] + w_up * G[j + 1];
                double e = S * X[2 * j - i + T] - K;
                int red = is_red(c, e);
                double gap = (isfinite(c) && isfinite(e)) ? (c - e) / K : -INFINITY;
                G[j] = red ? c : e;
                last = red ? j : last;
                gap_last = red ? gap : gap_last;
                gap_next = (!red && prev_red) ? -gap : gap_next; /* the cell after a red one */
                prev_red = red;
            }
        }
        if (boundary) boundary[i] = american ? last : (every == 0 ? -1 : i);
        if (margin && american) {
            margin[2 * i] = last >= 0 ? gap_last : NAN;
            margin[2 * i + 1] = (last + 1 <= i) ? gap_next : NAN;
        } else if (margin && every > 1) {
            margin[2 * i] = NAN;
            margin[2 * i + 1] = NAN;
        }
    }
    *price = G[0];
    free(X); free(G); free(D);
    return OR_OK;
}

/*
 * Trinomial American or European call -- Sec. 3 and appendix A.1.
 * Row i has columns 0..2i; children of (i,j) are (i+1,j) (down), (i+1,j+1)
 * (same price) and (i+1,j+2) (up).  boundary/margin as for the binomial call.
 */
static int oracle_trinomial(double S, double K, double r, double q, double sigma, double E,
                            int64_t T, int american, double *price, int64_t *boundary,
                            double *margin)
{
    const double dt = E / (double)T;
    const double A = sigma * sqrt(2.0 * dt);          /* u = e^{A} */
    const double su = exp(0.5 * A), sd = exp(-0.5 * A); /* sqrt(u), sqrt(d) */
    const double g = exp(0.5 * (r - q) * dt);
    const double pu = ((g - sd) / (su - sd)) * ((g - sd) / (su - sd));
    const double pd = ((su - g) / (su - sd)) * ((su - g) / (su - sd));
    const double po = 1.0 - pu - pd;
    const double m = exp(-r * dt);
    if (!(pu > 0.0 && pd > 0.0 && po >= 0.0))
        return OR_EPROB;
    const double w_d = m * pd, w_o = m * po, w_u = m * pu;

    const int64_t W = 2 * T + 1;
    double *X = (double *)malloc(sizeof(double) * (size_t)(2 * T + 1)); /* X[k+T] = e^{k A} */
    double *G = (double *)malloc(sizeof(double) * (size_t)W);
    double *D = margin ? (double *)malloc(sizeof(double) * (size_t)W) : NULL;
    if (!X || !G || (margin && !D)) {
        free(X); free(G); free(D);
        return OR_ENOMEM;
    }
    for (int64_t k = -T; k <= T; ++k)
        X[k + T] = exp((double)k * A);

    int64_t last = -1;
    for (int64_t j = 0; j <= 2 * T; ++j) {
        double e = S * X[j - T + T] - K;
        int red = is_red(0.0, e);
        G[j] = red ? 0.0 : e;
        if (D) D[j] = 0.0 - e;
        if (red) last = j;
    }
    if (boundary) boundary[T] = last;
    if (margin) {
        margin[2 * T] = last >= 0 ? D[last] / K : NAN;
        margin[2 * T + 1] = (last + 1 <= 2 * T) ? -D[last + 1] / K : NAN;
    }

    double gap_last = NAN, gap_next = NAN; /* decision gaps at the last red cell and the next */
    for (int64_t i = T - 1; i >= 0; --i) {
        last = -1;
        if (!american) {
            for (int64_t j = 0; j <= 2 * i; ++j)
                G[j] = w_d * G[j] + w_o * G[j + 1] + w_u * G[j + 2];
        } else if (!D) {
            for (int64_t j = 0; j <= 2 * i; ++j) {
                double c = w_d * G[j] + w_o * G[j + 1] + w_u * G[j + 2];
                double e = S * X[j - i + T] - K;
                int red = (c >= e) & (c < INFINITY) & (e < INFINITY); /* is_red() */
                G[j] = red ? c : e;
                last = red ? j : last;
            }
        } else {
            int prev_red = 1; /* column -1 counts as red: with no red cell the next cell is column 0 */
            for (int64_t j = 0; j <= 2 * i; ++j) {
                double c = w_d * G[j] + w_o * G[j + 1] + w_u * G[j + 2];
                double e = S * X[j - i + T] - K;
                int red = is_red(c, e);
                double gap = (isfinite(c) && isfinite(e)) ? (c - e) / K : -INFINITY;
                G[j] = red ? c : e;
                last = red ? j : last;
                gap_last = red ? gap : gap_last;
                gap_next = (!red && prev_red) ? -gap : gap_next; /* the cell after a red one */
                prev_red = red;
            }
        }
        if (boundary) boundary[i] = american ? last : -1;
        if (margin && american) {
            margin[2 * i] = last >= 0 ? gap_last : NAN;
            margin[2 * i + 1] = (last + 1 <= 2 * i) ? gap_next : NAN;
        }
    }
    *price = G[0];
    free(X); free(G); free(D);
    return OR_OK;
}

/*
 * Black-Scholes-Merton American or European put -- Sec. 4.2, eq. (bsmG).
 * Grid v^n_k ~ v~(n dtau, s0 + k ds), n = 0..T, on the cone |k| <= T-n.
 * Green (exercise) iff g > continuation.  boundary[n] = last green k of step
 * n (INT64_MIN if none); margin[2n] = g-cont at it, margin[2n+1] = cont-g at
 * k+1 (nondimensional values, so the scale is 1).  The price is K * v^T_0.
 */
static int oracle_bsm_put(double S, double K, double r, double q, double sigma, double E,
                          int64_t T, int american, double lambda, double *price,
                          int64_t *boundary, double *margin)
{
    if (q != 0.0)
        return OR_EINVAL; /* the PDE of Sec. 4.1 carries no dividend term */
    const double dtau = 0.5 * sigma * sigma * E / (double)T;
    const double ds = sqrt(dtau / lambda);
    const double omega = 2.0 * r / (sigma * sigma);
    const double lam = dtau / (ds * ds);
    const double drift = 0.5 * (omega - 1.0) * dtau / ds;
    const double ca = lam + drift;                    /* weight on v_{k+1} */
    const double cb = lam - drift;                    /* weight on v_{k-1} */
    const double cc = 1.0 - omega * dtau - 2.0 * lam; /* weight on v_k     */
    if (!(ca >= 0.0 && cb >= 0.0 && cc >= 0.0))
        return OR_EPROB;
    const double s0 = log(S / K);

    const int64_t W = 2 * T + 1;
    double *EX = (double *)malloc(sizeof(double) * (size_t)W); /* EX[k+T] = e^{s0 + k ds} */
    double *V = (double *)malloc(sizeof(double) * (size_t)W);  /* step n-1 */
    double *Vn = (double *)malloc(sizeof(double) * (size_t)W); /* step n   */
    double *D = margin ? (double *)malloc(sizeof(double) * (size_t)W) : NULL;
    if (!EX || !V || !Vn || (margin && !D)) {
        free(EX); free(V); free(Vn); free(D);
        return OR_ENOMEM;
    }
    for (int64_t k = -T; k <= T; ++k)
        EX[k + T] = exp(s0 + (double)k * ds);

    /* Step 0 (expiry): v^0_k = max(1 - e^{s_k}, 0); exercise cells have g > 0. */
    int64_t lastg = INT64_MIN;
    for (int64_t k = -T; k <= T; ++k) {
        double g = 1.0 - EX[k + T];
        int green = g > 0.0;
        V[k + T] = green ? g : 0.0;
        if (D) D[k + T] = g;
        if (green) lastg = k;
    }
    if (boundary) boundary[0] = lastg;
    if (margin) {
        margin[0] = lastg != INT64_MIN ? D[lastg + T] : NAN;
        margin[1] = (lastg != INT64_MIN && lastg + 1 <= T) ? -D[lastg + 1 + T] : NAN;
    }

    double gap_last = NAN, gap_next = NAN; /* decision gaps at the last green cell and the next */
    for (int64_t n = 1; n <= T; ++n) {
        const int64_t lo = -(T - n), hi = T - n;
        lastg = INT64_MIN;
        if (!american) {
            for (int64_t k = lo; k <= hi; ++k)
                Vn[k + T] = cb * V[k - 1 + T] + cc * V[k + T] + ca * V[k + 1 + T];
        } else if (!D) {
            for (int64_t k = lo; k <= hi; ++k) {
                double cont = cb * V[k - 1 + T] + cc * V[k + T] + ca * V[k + 1 + T];
                double g = 1.0 - EX[k + T];
                int green = g > cont;
                Vn[k + T] = green ? g : cont;
                lastg = green ? k : lastg;
            }
        } else {
            int prev_green = 0;
            for (int64_t k = lo; k <= hi; ++k) {
                double cont = cb * V[k - 1 + T] + cc * V[k + T] + ca * V[k + 1 + T];
                double g = 1.0 - EX[k + T];
                int green = g > cont;
                Vn[k + T] = green ? g : cont;
                lastg = green ? k : lastg;
                gap_last = green ? g - cont : gap_last;
                gap_next = (!green && prev_green) ? cont - g : gap_next; /* the cell after a green one */
                prev_green = green;
            }
        }
        if (boundary) boundary[n] = american ? lastg : INT64_MIN;
        if (margin && american) {
            margin[2 * n] = lastg != INT64_MIN ? gap_last : NAN;
            margin[2 * n + 1] = (lastg != INT64_MIN && lastg + 1 <= hi) ? gap_next : NAN;
        }
        double *t = V; V = Vn; Vn = t;
    }
    *price = K * V[0 + T];
    free(EX); free(V); free(Vn); free(D);
    return OR_OK;
}

/*
 * European call on the binomial or trinomial lattice as a sum over the
 * distribution of the number of up moves (the closed form of the linear
 * stencil's T-fold application that the paper's European section evaluates
 * with one FFT): price = disc * sum_k P(k) (S e^{(2k-n) h} - K)^+, with
 * P(k) = C(n,k) p^k (1-p)^{n-k}.
 *   binomial:  n = T, p of Fig. 1, h = a = V sqrt(dt), disc = m^T.
 *   trinomial: a trinomial step with p_u = alpha^2, p_o = 2 alpha (1-alpha),
 *              p_d = (1-alpha)^2 (Sec. 3) is two half steps of +-A/2 that go
 *              up with probability alpha, so after T steps the position is
 *              binomial over n = 2T half steps: p = alpha, h = A/2,
 *              disc = m^T.
 * P(k) is built from ratios of consecutive terms outward from the mode and
 * normalised by its sum (no lgamma cancellation at large n).  O(n) work.
 */
static int european_sum(double S, double K, double p, double h, int64_t n, double disc, double *price)
{
    double *w = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    if (!w)
        return OR_ENOMEM;
    int64_t mode = (int64_t)floor((double)(n + 1) * p);
    if (mode > n) mode = n;
    if (mode < 0) mode = 0;
    const double odds = p / (1.0 - p);
    w[mode] = 1.0;
    for (int64_t k = mode + 1; k <= n; ++k)
        w[k] = w[k - 1] * ((double)(n - k + 1) / (double)k) * odds;
    for (int64_t k = mode - 1; k >= 0; --k)
        w[k] = w[k + 1] * ((double)(k + 1) / (double)(n - k)) / odds;
    double z = 0.0, acc = 0.0;
    for (int64_t k = 0; k <= n; ++k) {
        z += w[k];
        double pay = S * exp((double)(2 * k - n) * h) - K;
        if (pay > 0.0 && isfinite(pay))
            acc += w[k] * pay;
        else if (pay > 0.0 && w[k] > 0.0)
            acc = INFINITY;
    }
    free(w);
    *price = disc * (acc / z);
    return OR_OK;
}

int aop_oracle_european_sum(int model, double S, double K, double r, double q, double sigma, double E,
                            int64_t T, double *price)
{
    if (!price)
        return OR_EINVAL;
    if (!(isfinite(S) && isfinite(K) && isfinite(r) && isfinite(q) && isfinite(sigma) &&
          isfinite(E)) ||
        S <= 0.0 || K <= 0.0 || sigma <= 0.0 || E <= 0.0 || T < 1 || q < 0.0)
        return OR_EINVAL;
    const double dt = E / (double)T;
    const double m = exp(-r * dt);
    const double disc = pow(m, (double)T);
    if (model == OR_BINOMIAL) {
        const double a = sigma * sqrt(dt);
        const double u = exp(a), d = 1.0 / u;
        const double p = (exp((r - q) * dt) - d) / (u - d);
        if (!(p > 0.0 && p < 1.0))
            return OR_EPROB;
        return european_sum(S, K, p, a, T, disc, price);
    }
    if (model == OR_TRINOMIAL) {
        const double A = sigma * sqrt(2.0 * dt);
        const double su = exp(0.5 * A), sd = exp(-0.5 * A);
        const double g = exp(0.5 * (r - q) * dt);
        const double alpha = (g - sd) / (su - sd);
        if (!(alpha > 0.0 && alpha < 1.0))
            return OR_EPROB;
        return european_sum(S, K, alpha, 0.5 * A, 2 * T, disc, price);
    }
    return OR_EINVAL;
}

/*
 * Gaussian approximations of the European binomial call (the paper's section
 * on the European call under the binomial model): the number of up moves x of
 * the T-step lattice is approximated by a normal density with mean pT and
 * variance v = p(1-p)T, so that
 *   price ~ m^T / sqrt(2 pi v) * sum_x (S u^{2x-T} - K)^+ e^{-(x - pT)^2 / (2v)}.
 * method 0: the sum over x in [max(pT - 6 sqrt v, 0), min(pT + 6 sqrt v, T) - 1]
 *           (x integer, the window bounds rounded up), O(sqrt T) terms;
 * method 1: the sum over x in [0, T-1], O(T) terms;
 * method 2: the integral of the same density times (S u^{2x-T} - K) from
 *           x0 = ceil(T/2 + ln(K/S) / (2 ln u)) to T, in closed form with erf:
 *           m^T/2 [ S u^{2(v ln u + pT) - T} erf((x - pT)/sqrt(2v) - ln u sqrt(2v))
 *                   - K erf((x - pT)/sqrt(2v)) ] from x0 to T, O(1).
 * (The paper writes the mean as -pT inside (x + mu); the same density.)
 */
int aop_oracle_european_gauss(int method, double S, double K, double r, double q, double sigma, double E,
                              int64_t T, double *price)
{
    if (!price || method < 0 || method > 2)
        return OR_EINVAL;
    if (!(isfinite(S) && isfinite(K) && isfinite(r) && isfinite(q) && isfinite(sigma) &&
          isfinite(E)) ||
        S <= 0.0 || K <= 0.0 || sigma <= 0.0 || E <= 0.0 || T < 1 || q < 0.0)
        return OR_EINVAL;
    const double dt = E / (double)T;
    const double a = sigma * sqrt(dt); /* ln u */
    const double u = exp(a), d = 1.0 / u;
    const double p = (exp((r - q) * dt) - d) / (u - d);
    const double m = exp(-r * dt);
    if (!(p > 0.0 && p < 1.0))
        return OR_EPROB;
    const double mu = p * (double)T;
    const double v = p * (1.0 - p) * (double)T;
    const double disc = pow(m, (double)T);
    if (method == 2) {
        const double x0 = ceil(0.5 * (double)T + log(K / S) / (2.0 * a));
        const double lo = x0 > (double)T ? (double)T : x0;
        const double sv2 = sqrt(2.0 * v);
        const double gS = S * exp((2.0 * (v * a + mu) - (double)T) * a);
        const double sterm = gS * (erf(((double)T - mu) / sv2 - a * sv2) - erf((lo - mu) / sv2 - a * sv2));
        const double kterm = K * (erf(((double)T - mu) / sv2) - erf((lo - mu) / sv2));
        *price = 0.5 * disc * (sterm - kterm);
        return OR_OK;
    }
    int64_t xlo = 0, xhi = T - 1;
    if (method == 0) {
        const double sd = sqrt(v);
        const double lo = ceil(mu - 6.0 * sd), hi = ceil(mu + 6.0 * sd);
        xlo = lo > 0.0 ? (int64_t)lo : 0;
        xhi = (hi < (double)T ? (int64_t)hi : T) - 1;
    }
    double acc = 0.0;
    for (int64_t x = xlo; x <= xhi; ++x) {
        const double pay = S * exp((double)(2 * x - T) * a) - K;
        if (pay > 0.0)
            acc += pay * exp(-((double)x - mu) * ((double)x - mu) / (2.0 * v));
    }
    *price = disc * acc / sqrt(2.0 * M_PI * v);
    return OR_OK;
}

/*
 * Entry point.  model: 0 binomial call, 1 trinomial call, 2 BSM put.
 * boundary: NULL or T+1 entries; margin: NULL or 2(T+1) entries.
 * lambda: dtau/ds^2 for the BSM grid (ignored otherwise).
 * Returns 0 on success, 1 for invalid arguments, 2 when the lattice
 * probabilities or scheme coefficients leave [0,1], 3 when out of memory.
 */
int aop_oracle_price(int model, double S, double K, double r, double q, double sigma,
                     double E, int64_t T, int american, double lambda, double *price,
                     int64_t *boundary, double *margin)
{
    /* american: 1 American, 0 European; for the binomial call d >= 2 prices
     * the Bermudan call exercisable every d steps back from expiry. */
    if (american < 0 || (american > 1 && model != OR_BINOMIAL))
        return OR_EINVAL;
    if (!price)
        return OR_EINVAL;
    if (!(isfinite(S) && isfinite(K) && isfinite(r) && isfinite(q) && isfinite(sigma) &&
          isfinite(E)) ||
        S <= 0.0 || K <= 0.0 || sigma <= 0.0 || E <= 0.0 || T < 1 || q < 0.0)
        return OR_EINVAL;
    switch (model) {
    case OR_BINOMIAL:
        return oracle_binomial(S, K, r, q, sigma, E, T, (int64_t)american, price, boundary, margin);
    case OR_TRINOMIAL:
        return oracle_trinomial(S, K, r, q, sigma, E, T, american, price, boundary, margin);
    case OR_BSM_PUT:
        if (!(lambda > 0.0 && lambda <= 0.5))
            return OR_EINVAL;
        return oracle_bsm_put(S, K, r, q, sigma, E, T, american, lambda, price, boundary, margin);
    default:
        return OR_EINVAL;
    }
}
