// aop_cpu.cpp -- the FFT nonlinear-stencil method on host cores (OpenMP
// tasks), the paper's own setting: a multicore implementation of the same
// recursion as the GPU library, for comparison with it and with the plain
// induction.  Not a fallback of the GPU path: a separate library with its own
// entry points (include/aop_cpu.h).
//
// Method (Sec. 2.3 binomial, Sec. 3 trinomial, Sec. 4.3 BSM): the expiry row
// and the row below it are computed directly; the red (continuation) region is
// cut into trapezoids ("Partitioning the triangle"), each solved recursively
// ("Solving a trapezoid"): the left part of a trapezoid is advanced h1 rows by
// one correlation with the h1-step stencil kernel (computed by FFT, or by
// stepping the linear stencil when that is cheaper) while the sub-trapezoid at
// the boundary is solved as a task; then the same for the lower half.  Leaves
// of at most `base` red cells are stepped directly with the max(continuation,
// exercise) stencil of Def. 2.1 / eq. bsmG.  The FFT is an iterative radix-2
// transform whose butterfly loops become OpenMP tasks for long transforms.
#include <omp.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "aop.h"
#include "aop_cpu.h"

namespace {

typedef std::complex<double> cd;
typedef int64_t ll;

constexpr int BINOMIAL = 0, TRINOMIAL = 1, BSM = 2;
constexpr ll NONE = INT64_MIN;

// ------------------------------------------------------------------ FFT
// Twiddles e^{-2 pi i t / N}, t < N/2, per transform size (built once).
struct Twiddles {
    std::once_flag once[32];
    std::vector<cd> w[32];
    const cd *get(int lg)
    {
        std::call_once(once[lg], [&] {
            const ll N = ll(1) << lg;
            w[lg].resize((size_t)std::max<ll>(N / 2, 1));
            for (ll t = 0; t < N / 2; ++t) {
                const double ang = -2.0 * M_PI * (double)t / (double)N;
                w[lg][(size_t)t] = cd(std::cos(ang), std::sin(ang));
            }
        });
        return w[lg].data();
    }
};
Twiddles g_tw;

constexpr int PAR_LG = 15;  // transforms of at least 2^15 points run their stages as tasks

// In-place radix-2 transform of 2^lg points; inverse = conjugate twiddles,
// unscaled.  Bit-reversal permutation, then log2 N butterfly stages.
void fft(cd *x, int lg, bool inverse)
{
    const ll N = ll(1) << lg;
    for (ll i = 1, j = 0; i < N; ++i) {
        ll bit = N >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(x[i], x[j]);
    }
    const cd *tw = g_tw.get(lg);
    for (int s = 1; s <= lg; ++s) {
        const ll L = ll(1) << s, half = L >> 1, stride = N / L;
        auto body = [&](ll q) {  // butterfly q of N/2: block q / half, offset q % half
            const ll blk = q / half, k = q % half;
            const cd w = tw[k * stride];
            const double wr = w.real(), wi = inverse ? -w.imag() : w.imag();
            cd *a = x + blk * L + k;
            const double br = a[half].real(), bi = a[half].imag();
            const double tr = wr * br - wi * bi, ti = wr * bi + wi * br;  // plain product, no NaN rescue
            const double ar = a[0].real(), ai = a[0].imag();
            a[half] = cd(ar - tr, ai - ti);
            a[0] = cd(ar + tr, ai + ti);
        };
        if (lg >= PAR_LG) {
#pragma omp taskloop grainsize(4096)
            for (ll q = 0; q < N / 2; ++q) body(q);
        } else {
            for (ll q = 0; q < N / 2; ++q) body(q);
        }
    }
}

// ------------------------------------------------------------- option
struct Opt {
    int model;
    bool no_green, european;
    ll T;
    double S, K, a, s0, w0, w1, w2;
};

double ex_bin(const Opt &d, ll i, ll j) { return d.S * std::exp((double)(2 * j - i) * d.a) - d.K; }
double ex_tri(const Opt &d, ll i, ll j) { return d.S * std::exp((double)(j - i) * d.a) - d.K; }
double ex_lat(const Opt &d, ll i, ll j) { return d.model == BINOMIAL ? ex_bin(d, i, j) : ex_tri(d, i, j); }
double ex_bsm(const Opt &d, ll k) { return 1.0 - std::exp(d.s0 + (double)k * d.a); }
bool red_of(double c, double e) { return c >= e && c < INFINITY && e < INFINITY; }

// h-step kernel spectrum at theta = 2 pi f / N in polar form (FP64): |P|^2 =
// rho^2 (1 + delta) from s = sin^2(theta/2), magnitude by log1p, phase by atan2.
// beta tilts the one-step weights by e^{beta k}.
cd kernel_power(const Opt &d, double h, ll f, ll N, double beta)
{
    const double x = (double)(f <= N / 2 ? f : f - N) / (double)N;
    const double sh = std::sin(M_PI * x), s = sh * sh;
    const double sn = std::sin(2.0 * M_PI * x), cs = std::cos(2.0 * M_PI * x);
    double rho, delta, arg;
    if (d.model == BINOMIAL) {
        const double wd = d.w0, wu = d.w1 * (beta != 0.0 ? std::exp(beta) : 1.0);
        rho = wd + wu;
        delta = -4.0 * wd * wu * s / (rho * rho);
        arg = std::atan2(wu * sn, wd + wu * cs);
    } else {
        const double wm = d.w0 * (beta != 0.0 ? std::exp(-beta) : 1.0), wc = d.w1;
        const double wp = d.w2 * (beta != 0.0 ? std::exp(beta) : 1.0);
        rho = wm + wc + wp;
        const double sp = wp + wm, df = wp - wm;
        delta = (-4.0 * s * (rho * sp - df * df) + 16.0 * wp * wm * s * s) / (rho * rho);
        arg = std::atan2(df * sn, rho - 2.0 * sp * s);
    }
    const double lrel = 0.5 * h * std::log1p(delta);
    if (!(lrel > -60.0)) return cd(0.0, 0.0);
    return std::polar(std::exp(h * std::log(rho) + lrel), h * arg);
}

int span_of(const Opt &d) { return d.model == BINOMIAL ? 1 : 2; }

// dst[t] = (x (*) W^h)[out_off + t], t < n_out, x = src[0 .. n_in): the
// correlation with the h-step kernel (binomial one-sided, offsets 0..h;
// trinomial / BSM centred, offsets -h..h).  With beta != 0 the input is tilted
// by e^{-beta (t - tc)} and the output untilted by e^{beta (m - tc)}.
// P(theta_f)^h for the bins f = 0 .. N/2 of a 2^lg-point transform (real
// input: the other bins are their conjugates).
void fill_spectrum(const Opt &d, double h, int lg, double beta, cd *out)
{
    const ll N = ll(1) << lg;
    if (lg >= PAR_LG) {
#pragma omp taskloop grainsize(4096)
        for (ll f = 0; f <= N / 2; ++f) out[f] = kernel_power(d, h, f, N, beta);
    } else {
        for (ll f = 0; f <= N / 2; ++f) out[f] = kernel_power(d, h, f, N, beta);
    }
}

// Kernel spectra of one option keyed by (h, log2 N): the frames of one
// recursion level share their heights, so each spectrum is evaluated once.
struct SpectrumCache {
    struct Entry {
        std::once_flag once;
        std::vector<cd> p;
    };
    std::mutex mu;
    std::vector<std::pair<std::pair<ll, int>, Entry *>> keys;
    ~SpectrumCache()
    {
        for (auto &k : keys) delete k.second;
    }
    const cd *get(const Opt &d, ll h, int lg, double beta)
    {
        if (beta != 0.0) return nullptr;  // tilted spectra are used once
        Entry *e = nullptr;
        {
            std::lock_guard<std::mutex> g(mu);
            for (auto &k : keys)
                if (k.first.first == h && k.first.second == lg) e = k.second;
            if (!e) {
                e = new Entry;
                keys.push_back({{h, lg}, e});
            }
        }
        std::call_once(e->once, [&] {
            e->p.resize((size_t)((ll(1) << (lg - 1)) + 1));
            fill_spectrum(d, (double)h, lg, 0.0, e->p.data());
        });
        return e->p.data();
    }
};

void correlate(const Opt &d, const double *src, ll n_in, ll h, ll out_off, ll n_out, double *dst,
               double beta = 0.0, double tc = 0.0, SpectrumCache *cache = nullptr)
{
    if (n_out <= 0) return;
    const int sp = span_of(d);
    int lg = 1;
    while ((ll(1) << lg) < n_in) ++lg;
    const ll N = ll(1) << lg;
    const double direct_cost = 3.0 * (double)n_in * (double)h;
    const double fft_cost = (double)N * (10.0 * lg + 60.0);
    if (beta == 0.0 && direct_cost <= fft_cost) {
        // h steps of the linear stencil, left-aligned: z'_j = sum_s w_s z_{j+s}
        std::vector<double> z(src, src + n_in);
        ll len = n_in;
        for (ll k = 0; k < h; ++k) {
            len -= sp;
            if (sp == 1)
                for (ll j = 0; j < len; ++j) z[j] = d.w0 * z[j] + d.w1 * z[j + 1];
            else
                for (ll j = 0; j < len; ++j) z[j] = d.w0 * z[j] + d.w1 * z[j + 1] + d.w2 * z[j + 2];
        }
        const ll shift = (sp == 1) ? out_off : out_off - h;  // centred kernels start at offset -h
        for (ll t = 0; t < n_out; ++t) dst[t] = z[shift + t];
        return;
    }
    // Real input of N points as N/2 complex points z_t = x_{2t} + i x_{2t+1}:
    // one half-length transform, unpacked to the bins 0..N/2 of x.
    const ll M = N / 2;
    std::vector<cd> z((size_t)M, cd(0.0, 0.0));
    auto in = [&](ll t) {
        if (t >= n_in) return 0.0;
        double v = src[t];
        if (!(v < INFINITY)) return 0.0;  // an overflowed row value carries no weight (see the GPU path)
        if (beta != 0.0 && v != 0.0) v *= std::exp(-beta * ((double)t - tc));
        return v;
    };
    for (ll t = 0; t < M; ++t) z[(size_t)t] = cd(in(2 * t), in(2 * t + 1));
    fft(z.data(), lg - 1, false);
    const cd *P = cache ? cache->get(d, h, lg, beta) : nullptr;
    std::vector<cd> own;
    if (!P) {
        own.resize((size_t)(M + 1));
        fill_spectrum(d, (double)h, lg, beta, own.data());
        P = own.data();
    }
    const cd *tw = g_tw.get(lg);  // e^{-2 pi i f / N}, f < N/2
    std::vector<cd> zo((size_t)M);
    for (ll f = 0; f <= M / 2; ++f) {  // bins f and M - f together
        const ll g = (M - f) % M;
        const cd Zf = z[(size_t)f], Zg = z[(size_t)g];
        auto bin = [&](const cd &Za, const cd &Zb, ll k) {  // X_k from Z_k, Z_{M-k}
            const cd A = 0.5 * (Za + std::conj(Zb)), Bm = 0.5 * (Za - std::conj(Zb));
            const cd B(Bm.imag(), -Bm.real());  // Bm / i
            const cd w = (k < M) ? tw[k] : cd(-1.0, 0.0);
            const cd wB(w.real() * B.real() - w.imag() * B.imag(), w.real() * B.imag() + w.imag() * B.real());
            return A + wB;
        };
        cd Xf = bin(Zf, Zg, f), Xg = bin(Zg, Zf, M - f);
        cd Xh = (f == 0) ? bin(Zf, Zg, M) : Xg;  // f = 0: the Nyquist bin M
        auto mul = [](const cd &a, const cd &b) {
            return cd(a.real() * b.real() - a.imag() * b.imag(), a.real() * b.imag() + a.imag() * b.real());
        };
        const cd Yf = mul(Xf, P[f]);
        const cd Yg = mul(Xh, P[f == 0 ? M : M - f]);
        // pack back: Z'_k = (Y_k + conj(Y_{M-k})) + i e^{2 pi i k / N} (Y_k - conj(Y_{M-k}))
        auto pack = [&](const cd &Ya, const cd &Yb, ll k) {
            const cd E = Ya + std::conj(Yb), Om = Ya - std::conj(Yb);
            const cd w = std::conj(k < M ? tw[k] : cd(-1.0, 0.0));
            const cd O(w.real() * Om.real() - w.imag() * Om.imag(), w.real() * Om.imag() + w.imag() * Om.real());
            return E + cd(-O.imag(), O.real());
        };
        zo[(size_t)f] = pack(Yf, Yg, f);
        if (g != f && f != 0) zo[(size_t)g] = pack(Yg, Yf, g);
    }
    fft(zo.data(), lg - 1, true);
    const double invN = 1.0 / (double)N;
    for (ll t = 0; t < n_out; ++t) {
        const ll m = out_off + t;
        const cd &q = zo[(size_t)(m >> 1)];
        double y = ((m & 1) ? q.imag() : q.real()) * invN;
        if (beta != 0.0) y *= std::exp(beta * ((double)m - tc));
        dst[t] = y;
    }
}

// ------------------------------------------------------------- solver
struct Solver {
    Opt d;
    SpectrumCache spc;
    int base;      // leaves: at most this many red cells
    ll task_min;   // correlations of at least this many cells run as tasks
    ll *bnd;       // T+1 entries or nullptr

    void note(ll row, ll v)
    {
        if (bnd) bnd[row] = v;
    }

    // Lattice leaf: rows i0-1 .. i0-h from row i0 (red cells [c0, b] in src,
    // absolute column indices), columns >= c0 only; writes the red cells of row
    // i0-h to dst and returns its boundary; *v0 = value of column c0 there.
    ll band_lat(ll i0, ll c0, ll h, ll b, const double *src, double *dst, double *v0)
    {
        const int sp = span_of(d);
        const double u = std::exp(d.a);
        const ll wr = (sp == 1) ? 1 : 2;  // last column of row i: wr * i
        const ll W = (b - c0 + 1) + sp;   // red cells plus the green cells they read
        std::vector<double> g((size_t)std::max<ll>(W, 1)), x((size_t)std::max<ll>(W, 1));
        auto seed = [&](ll i) {  // S u^{cs j - i} of the band's columns at row i
            for (ll q = 0; q < W; ++q) {
                const ll j = c0 + q;
                x[(size_t)q] = (sp == 1) ? d.S * std::exp((double)(2 * j - i) * d.a) : d.S * std::exp((double)(j - i) * d.a);
            }
        };
        seed(i0);
        for (ll q = 0; q < W; ++q) {
            const ll j = c0 + q;
            g[(size_t)q] = (j <= b) ? src[j] : (j <= wr * i0 ? x[(size_t)q] - d.K : 0.0);
        }
        ll bc = b;
        for (ll k = 1; k <= h; ++k) {
            const ll i = i0 - k;
            // exercise values of row i+1 beyond the red cells feed the last red cells
            const ll jmax = std::min(bc, wr * i);  // red cells of row i lie in [c0, bc]
            ll last = c0 - 1;
            for (ll j = c0; j <= jmax; ++j) {
                const ll q = j - c0;
                double c = d.w0 * g[(size_t)q] + d.w1 * g[(size_t)q + 1];
                if (sp == 2) c += d.w2 * g[(size_t)q + 2];
                const double e = x[(size_t)q] * u - d.K;  // S u^{.} one row lower
                const bool red = red_of(c, e);
                g[(size_t)q] = red ? c : e;
                if (red) last = j;
            }
            for (ll q = 0; q < W; ++q) x[(size_t)q] *= u;
            if ((k & 31) == 0) seed(i);  // re-seed the carried exponentials
            for (ll j = std::max(jmax + 1, c0); j < c0 + W; ++j)  // green: exercise values
                g[(size_t)(j - c0)] = (j <= wr * i) ? x[(size_t)(j - c0)] - d.K : 0.0;
            bc = last;
            note(i, bc);
        }
        for (ll j = c0; j <= bc; ++j) dst[j] = g[(size_t)(j - c0)];
        if (v0) *v0 = g[0];
        return bc;
    }

    // solve(i0, c0, h, b): red cells [c0, b] of row i0 in src -> row i0-h in dst.
    ll solve_lat(ll i0, ll c0, ll h, ll b, const double *src, double *dst)
    {
        const int sp = span_of(d);
        const ll nred = b - c0 + 1;
        if (nred <= base) return band_lat(i0, c0, h, b, src, dst, nullptr);
        const ll h1 = h / 2, h2 = h - h1;
        std::vector<double> midv((size_t)(nred + 1));
        double *mid = midv.data() - c0;  // absolute column indexing
        // (1) the left part of row i0-h1 by one correlation, while (2) the
        // sub-trapezoid at the boundary produces the rest of that row
        const ll n1 = nred - sp * h1;
#pragma omp task if (nred >= task_min) default(shared) firstprivate(c0, nred, h1, n1)
        correlate(d, src + c0, nred, h1, sp == 1 ? 0 : h1, n1, mid + c0, 0.0, 0.0, &spc);
        const ll br = solve_lat(i0, b - sp * h1 + 1, h1, b, src, mid);
#pragma omp taskwait
        const ll n2 = br - c0 + 1;
        if (n2 - sp * h2 > 0) {
#pragma omp task if (n2 >= task_min) default(shared) firstprivate(c0, n2, h2)
            correlate(d, mid + c0, n2, h2, sp == 1 ? 0 : h2, n2 - sp * h2, dst + c0, 0.0, 0.0, &spc);
        }
        const ll bo = solve_lat(i0 - h1, br - sp * h2 + 1, h2, br, mid, dst);
#pragma omp taskwait
        return bo;
    }

    double drive_lattice()
    {
        const ll T = d.T;
        const int sp = span_of(d);
        const ll wT = (sp == 1) ? T : 2 * T;
        std::vector<double> A((size_t)(wT + 3)), B((size_t)(wT + 3));
        std::vector<double> gT((size_t)(wT + 1));
        ll lastT = -1;
        for (ll j = 0; j <= wT; ++j) {
            const double e = ex_lat(d, T, j);
            const bool red = red_of(0.0, e);
            gT[(size_t)j] = red ? 0.0 : e;
            if (red) lastT = j;
        }
        note(T, lastT);
        const ll w1 = wT - sp;
        ll b = -1;
        for (ll j = 0; j <= w1; ++j) {
            double c = d.w0 * gT[(size_t)j] + d.w1 * gT[(size_t)j + 1];
            if (sp == 2) c += d.w2 * gT[(size_t)j + 2];
            const double e = ex_lat(d, T - 1, j);
            const bool red = d.european || red_of(c, e);
            A[(size_t)j] = red ? c : e;
            if (red) b = j;
        }
        note(T - 1, d.european ? -1 : b);
        if (T > 1 && (b == w1 || d.no_green || d.european)) {
            // no exercise below row T-1 (Lemma 2.3 with Y = 0, an entirely red
            // row, or a European option): one tilted correlation to the root
            if (bnd)
                for (ll i = 0; i < T - 1; ++i) bnd[i] = d.european ? -1 : (sp == 1 ? i : 2 * i);
            note(T - 1, d.european ? -1 : w1);
            const double beta = (sp == 1) ? 2.0 * d.a : d.a;
            double tc = (sp == 1) ? 0.5 * ((double)(T - 1) + std::log(d.K / d.S) / d.a)
                                  : (double)(T - 1) + std::log(d.K / d.S) / d.a;
            tc = std::min(std::max(tc, 0.0), (double)w1);
            double root = 0.0;
            correlate(d, A.data(), w1 + 1, T - 1, sp == 1 ? 0 : T - 1, 1, &root, beta, tc);
            return root;
        }
        ll i0 = T - 1;
        double *src = A.data(), *dst = B.data();
        while (i0 > 0) {
            if (b < 0) {  // no red cell: every row below is green (Lemma 2.4)
                for (ll i = 0; i < i0; ++i) note(i, -1);
                return d.S - d.K;
            }
            const ll nred = b + 1;
            if (nred <= base) {  // the leftover triangle
                double v0 = 0.0;
                band_lat(i0, 0, i0, b, src, dst, &v0);
                return v0;
            }
            ll h = (sp == 1) ? nred : nred / 2;
            h = std::min(h, i0);
            b = solve_lat(i0, 0, h, b, src, dst);
            i0 -= h;
            std::swap(src, dst);
        }
        return b >= 0 ? src[0] : d.S - d.K;
    }

    // BSM leaf: steps n+1 .. n+h from step n, whose red cells (f, R0] are in
    // src (absolute offsets k); green (exercise) to the left.  Writes step
    // n+h's red cells up to R0-h to dst; returns its boundary; *vr = value of
    // cell R0-h there.
    ll band_bsm(ll n0, ll f, ll h, ll R0, const double *src, double *dst, double *vr)
    {
        const ll T = d.T;
        const ll lo = f - h - 1;  // leftmost cell read: the boundary drops at most one per step
        const ll W = R0 - lo + 1;
        std::vector<double> v((size_t)W), vn((size_t)W), g((size_t)W);
        for (ll q = 0; q < W; ++q) {
            const ll k = lo + q;
            g[(size_t)q] = ex_bsm(d, k);
            v[(size_t)q] = (k > f) ? src[k] : g[(size_t)q];
        }
        ll fc = f;
        for (ll t = 1; t <= h; ++t) {
            const ll R = R0 - t;
            const ll kmin = std::max(fc, lo + 1);  // cells left of the old boundary stay green
            ll lastg = fc - 1;
            for (ll k = lo; k < kmin; ++k) vn[(size_t)(k - lo)] = g[(size_t)(k - lo)];
            for (ll k = kmin; k <= R; ++k) {
                const ll q = k - lo;
                const double cont = d.w0 * v[(size_t)q - 1] + d.w1 * v[(size_t)q] + d.w2 * v[(size_t)q + 1];
                const bool green = g[(size_t)q] > cont;
                vn[(size_t)q] = green ? g[(size_t)q] : cont;
                if (green) lastg = k;
            }
            std::swap(v, vn);
            fc = lastg;
            const ll n = n0 + t;
            note(n, fc < -(T - n) ? NONE : std::min(fc, T - n));
        }
        for (ll k = fc + 1; k <= R0 - h; ++k) dst[k] = v[(size_t)(k - lo)];
        if (vr) *vr = v[(size_t)(R0 - h - lo)];
        return fc;
    }

    // B(n, f, h): step n's red cells [f+1, f+2h] in src -> step n+h on
    // [f-h, f+h] in dst (the sub-trapezoid centred on the boundary f).
    ll solve_bsm(ll n, ll f, ll h, const double *src, double *dst)
    {
        if (2 * h <= base) return band_bsm(n, f, h, f + 2 * h, src, dst, nullptr);
        const ll h1 = h / 2, h2 = h - h1;
        const ll mlo = f - h1 + 1, mhi = f + h + h2;
        std::vector<double> midv((size_t)(mhi - mlo + 2));
        double *mid = midv.data() - mlo;
#pragma omp task if (2 * h >= task_min) default(shared) firstprivate(f, h, h1)
        correlate(d, src + f + 1, 2 * h, h1, h1, 2 * h - 2 * h1, mid + f + 1 + h1, 0.0, 0.0, &spc);
        const ll fp = solve_bsm(n, f, h1, src, mid);
#pragma omp taskwait
        const ll nin = f + h + h2 - fp;
#pragma omp task if (nin >= task_min) default(shared) firstprivate(fp, nin, h2)
        correlate(d, mid + fp + 1, nin, h2, h2, nin - 2 * h2, dst + fp + 1 + h2, 0.0, 0.0, &spc);
        const ll fo = solve_bsm(n + h1, fp, h2, mid, dst);
#pragma omp taskwait
        return fo;
    }

    double drive_bsm()
    {
        const ll T = d.T;
        const ll len = 3 * T + 3;  // k in [-2T-1, T+1]
        std::vector<double> Av((size_t)len), Bv((size_t)len);
        double *A = Av.data() + 2 * T + 1, *B = Bv.data() + 2 * T + 1;
        ll f0 = NONE, f1 = NONE;
        for (ll k = -T; k <= T; ++k)
            if (ex_bsm(d, k) > 0.0) f0 = k;
        note(0, f0);
        for (ll k = -(T - 1); k <= T - 1; ++k) {
            const double gm = ex_bsm(d, k - 1), g = ex_bsm(d, k), gp = ex_bsm(d, k + 1);
            const double cont = d.w0 * std::max(gm, 0.0) + d.w1 * std::max(g, 0.0) + d.w2 * std::max(gp, 0.0);
            const bool green = !d.european && g > cont;
            A[k] = green ? g : cont;
            if (green) f1 = k;
        }
        if (T >= 1) note(1, f1);
        ll n = 1, R = T - 1, L = -(T - 1);
        ll f = (f1 == NONE) ? L - 1 : f1;
        double *src = A, *dst = B;
        for (;;) {
            if (n == T) return d.K * ((f >= 0) ? ex_bsm(d, 0) : src[0]);
            if (f < L) {  // no exercise cell left in the cone: the rest is linear
                for (ll m = n + 1; m <= T; ++m) note(m, NONE);
                double v = 0.0;
                correlate(d, src + L, R - L + 1, T - n, T - n, 1, &v);
                return d.K * v;
            }
            if (f >= R) {  // the whole cone exercises, and keeps doing so
                for (ll m = n + 1; m <= T; ++m) note(m, T - m);
                return d.K * ex_bsm(d, 0);
            }
            const ll w = R - f;
            if (w <= base) {  // the leftover cone
                double vr = 0.0;
                band_bsm(n, f, T - n, R, src, dst, &vr);
                return d.K * vr;
            }
            const ll h = std::min(w / 2, T - n);
            // the red part right of the trapezoid, [f+1+h, R-h] of step n+h
#pragma omp task if (w >= task_min) default(shared) firstprivate(f, w, h)
            correlate(d, src + f + 1, w, h, h, w - 2 * h, dst + f + 1 + h, 0.0, 0.0, &spc);
            const ll fn = solve_bsm(n, f, h, src, dst);
#pragma omp taskwait
            n += h;
            R -= h;
            L += h;
            f = fn;
            std::swap(src, dst);
        }
    }
};

// Parameters of Fig. 1 (binomial), Sec. 3 (trinomial), eq. bsmG (BSM); the
// same validation as the GPU library's.
aop_status make_opt(const aop_option &o, double lambda, Opt &d)
{
    if (!(std::isfinite(o.S0) && std::isfinite(o.K) && std::isfinite(o.r) && std::isfinite(o.q) &&
          std::isfinite(o.sigma) && std::isfinite(o.expiry)))
        return AOP_EINVAL;
    if (o.S0 <= 0 || o.K <= 0 || o.sigma <= 0 || o.expiry <= 0 || o.q < 0 || o.T < 1 ||
        (o.flags & ~AOP_EUROPEAN) != 0 || o.exercise_every < 0)
        return AOP_EINVAL;
    if (o.exercise_every > 1) return AOP_ENOTIMPL;  // Bermudan exercise: the GPU library only
    if (o.T > AOP_MAX_T) return AOP_ETOOBIG;
    d = Opt{};
    d.model = o.model;
    d.T = o.T;
    d.S = o.S0;
    d.K = o.K;
    d.european = (o.flags & AOP_EUROPEAN) != 0;
    const double T = (double)o.T;
    if (o.model == AOP_BINOMIAL_CALL) {
        const double dt = o.expiry / T, a = o.sigma * std::sqrt(dt), u = std::exp(a), dn = 1.0 / u;
        const double p = (std::exp((o.r - o.q) * dt) - dn) / (u - dn), m = std::exp(-o.r * dt);
        if (!(p > 0.0 && p < 1.0)) return AOP_EPROB;
        d.a = a;
        d.w0 = m * (1.0 - p);
        d.w1 = m * p;
        d.no_green = o.q == 0.0 && o.r >= 0.0;
    } else if (o.model == AOP_TRINOMIAL_CALL) {
        const double dt = o.expiry / T, A = o.sigma * std::sqrt(2.0 * dt);
        const double su = std::exp(0.5 * A), sd = std::exp(-0.5 * A), g = std::exp(0.5 * (o.r - o.q) * dt);
        const double pu = ((g - sd) / (su - sd)) * ((g - sd) / (su - sd));
        const double pd = ((su - g) / (su - sd)) * ((su - g) / (su - sd));
        const double po = 1.0 - pu - pd, m = std::exp(-o.r * dt);
        if (!(pu > 0.0 && pd > 0.0 && po >= 0.0)) return AOP_EPROB;
        if (o.r < 0.0 && !d.european) return AOP_EPROB;  // outside the Sec. 3 lemmas' hypotheses
        d.a = A;
        d.w0 = m * pd;
        d.w1 = m * po;
        d.w2 = m * pu;
        d.no_green = o.q == 0.0 && o.r >= 0.0;
    } else if (o.model == AOP_BSM_PUT) {
        if (o.q != 0.0) return AOP_EINVAL;
        if (!(lambda > 0.0 && lambda <= 0.5)) return AOP_EINVAL;
        const double dtau = 0.5 * o.sigma * o.sigma * o.expiry / T, ds = std::sqrt(dtau / lambda);
        const double omega = 2.0 * o.r / (o.sigma * o.sigma), lam = dtau / (ds * ds);
        const double drift = 0.5 * (omega - 1.0) * dtau / ds;
        const double ca = lam + drift, cb = lam - drift, cc = 1.0 - omega * dtau - 2.0 * lam;
        if (!(ca >= 0.0 && cb >= 0.0 && cc >= 0.0)) return AOP_EPROB;
        d.a = ds;
        d.s0 = std::log(o.S0 / o.K);
        d.w0 = cb;
        d.w1 = cc;
        d.w2 = ca;
    } else {
        return AOP_EINVAL;
    }
    return AOP_OK;
}

}  // namespace

extern "C" {

aop_status aop_cpu_price_batch(const aop_option *opts, int64_t n, int32_t threads, int32_t base, double lambda,
                               double *price, int32_t *status, int64_t *boundary, int64_t boundary_stride)
{
    if (n < 0 || (n > 0 && (!opts || !price))) return AOP_EINVAL;
    if (lambda == 0.0) lambda = 1.0 / 3.0;
    if (base <= 0) base = 8;
    if (base < 2 || base > 4096) return AOP_EINVAL;
    if (boundary) {
        int64_t tmax = 0;
        for (int64_t i = 0; i < n; ++i) tmax = std::max<int64_t>(tmax, opts[i].T);
        if (boundary_stride < tmax + 1) return AOP_EINVAL;
    }
    if (threads <= 0) threads = omp_get_max_threads();
    std::vector<Opt> ds((size_t)std::max<int64_t>(n, 1));
    for (int64_t i = 0; i < n; ++i) {
        const aop_status st = make_opt(opts[i], lambda, ds[(size_t)i]);
        if (status) status[i] = st;
        if (st != AOP_OK) {
            ds[(size_t)i].model = -1;
            price[i] = NAN;
        }
    }
#pragma omp parallel num_threads(threads)
#pragma omp single
    for (int64_t i = 0; i < n; ++i) {
        if (ds[(size_t)i].model < 0) continue;
#pragma omp task firstprivate(i) default(shared)
        {
            Solver sv;
            sv.d = ds[(size_t)i];
            sv.base = base;
            sv.task_min = 4096;
            sv.bnd = boundary ? boundary + i * boundary_stride : nullptr;
            price[i] = sv.d.model == BSM ? sv.drive_bsm() : sv.drive_lattice();
        }
    }
    return AOP_OK;
}

}  // extern "C"
