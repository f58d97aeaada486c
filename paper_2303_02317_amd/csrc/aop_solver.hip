// aop_solver.hip -- gfx950 kernels of the FFT nonlinear-stencil pricer.
//
// One workgroup (256 lanes, 4 wave64) prices one option.  It
//   1. computes the expiry row and the first backward row directly (the
//      corollary relating consecutive boundaries only holds below the top row),
//   2. runs the trapezoid decomposition (Sec. 2.3 "Partitioning the triangle",
//      Sec. 3 / appendix A.3, Sec. 4.3): each trapezoid is solved recursively
//      ("Solving a trapezoid"); guaranteed-continuation (red) segments are
//      advanced h rows at once by an FFT correlation with the h-step stencil
//      kernel, whose spectrum is evaluated per bin in closed form (FP64);
//   3. solves the base cases with a one-wave band walker that applies the
//      max(continuation, exercise) stencil directly, one lane per cell, and
//      finds each row's boundary with a wave ballot.
// The recursion runs on an explicit stack in LDS; control flow is uniform
// across the workgroup.  Every range a step touches is checked against the
// option's workspace first; a failed check records an error and prices NaN.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <math.h>
#include <stdint.h>

#include "aop_internal.h"

namespace aop {

#define WG 256
#define NLDS 2048  // complex doubles staged in LDS per FFT tile (32 KB)
#define LG_NLDS 11
#define MAXD 48    // recursion depth bound (log2 of 2^22 plus slack)
#define BAND 64    // cells held by the band walker (one per lane)

typedef long long ll;

// ------------------------------------------------------------ small helpers
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b)  // a * conj(b)
{
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ unsigned bitrev(unsigned v, int lg)
{
    return lg ? (__brev(v) >> (32 - lg)) : 0u;
}
__device__ __forceinline__ int ceil_log2(ll n)
{
    int l = 0;
    while ((ll(1) << l) < n) ++l;
    return l;
}

// Exercise (green) values, evaluated at need (never stored).
__device__ __forceinline__ double ex_bin(const Desc &d, ll i, ll j)
{
    return d.S * exp((double)(2 * j - i) * d.a) - d.K;  // S u^{2j-i} - K
}
__device__ __forceinline__ double ex_tri(const Desc &d, ll i, ll j)
{
    return d.S * exp((double)(j - i) * d.a) - d.K;  // S u^{j-i} - K
}
__device__ __forceinline__ double ex_bsm(const Desc &d, ll k)
{
    return 1.0 - exp(d.s0 + (double)k * d.a);  // 1 - e^{s_k}
}
// Red (continuation) test of Definition 2.1 with the non-finite guard.
__device__ __forceinline__ bool red_of(double c, double e)
{
    return (c >= e) && (c < INFINITY) && (e < INFINITY);
}

__device__ ll block_max(ll v, ll *sh)
{
    for (int o = 32; o > 0; o >>= 1) {
        ll w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    ll r = sh[0];
    for (int w = 1; w < WG / 64; ++w) r = sh[w] > r ? sh[w] : r;
    __syncthreads();
    return r;
}

// --------------------------------------------------------- LDS radix-2 FFT
// nb batched transforms of length 2^lg, stored contiguously in LDS.
// Forward: decimation in frequency, natural order in -> bit-reversed out.
__device__ void lds_dif(double2 *x, int lg, int nb, const double2 *__restrict__ tw)
{
    if (lg <= 0) return;
    const int n = 1 << lg, half = n >> 1, total = nb * half;
    for (int s = lg - 1; s >= 0; --s) {
        const int m = 1 << s;
        for (int t = threadIdx.x; t < total; t += WG) {
            const int b = t >> (lg - 1);
            const int loc = t & (half - 1);
            const int j = loc & (m - 1);
            const int a = b * n + ((loc >> s) << (s + 1)) + j;
            const double2 u = x[a], v = x[a + m];
            const double2 w = tw[(ll)j << (LG_TW - s - 1)];  // e^{-2 pi i j / 2m}
            x[a] = make_double2(u.x + v.x, u.y + v.y);
            x[a + m] = cmul(make_double2(u.x - v.x, u.y - v.y), w);
        }
        __syncthreads();
    }
}
// Inverse (unnormalised): decimation in time, bit-reversed in -> natural out.
__device__ void lds_dit_inv(double2 *x, int lg, int nb, const double2 *__restrict__ tw)
{
    if (lg <= 0) return;
    const int n = 1 << lg, half = n >> 1, total = nb * half;
    for (int s = 0; s < lg; ++s) {
        const int m = 1 << s;
        for (int t = threadIdx.x; t < total; t += WG) {
            const int b = t >> (lg - 1);
            const int loc = t & (half - 1);
            const int j = loc & (m - 1);
            const int a = b * n + ((loc >> s) << (s + 1)) + j;
            const double2 u = x[a];
            const double2 v = cmulc(x[a + m], tw[(ll)j << (LG_TW - s - 1)]);  // * e^{+2 pi i j / 2m}
            x[a] = make_double2(u.x + v.x, u.y + v.y);
            x[a + m] = make_double2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
}

// ------------------------------------------------- h-step kernel spectrum
// Correlation y_m = sum_t W_t x_{m+t} with the h-fold one-step stencil has
// DFT multiplier P(theta)^h, P(theta) = sum_t w_t e^{i t theta}.  Evaluated in
// polar form in FP64: |P|^2 as rho^2 (1 + delta) with delta computed from
// s = sin^2(theta/2) without cancellation, log1p for the magnitude and atan2
// for the phase, so the h-th power costs O(1) and carries ~sqrt-free error.
//   binomial:  P = w_dn + w_up e^{i theta}                  (one-sided, offsets 0, 1)
//   trinomial / BSM: P = w_m e^{-i theta} + w_c + w_p e^{i theta}  (centred)
//   An exponential tilt beta (used only where a red segment spans a huge
//   dynamic range) replaces the one-step weights w_t by w_t e^{beta t} and
//   adds lscale to the log-magnitude.
__device__ double2 kernel_power(const Desc &d, ll h, ll f, int lgN, double beta, double lscale)
{
    const ll N = ll(1) << lgN;
    const ll ff = (f <= N / 2) ? f : f - N;
    const double x = (double)ff / (double)N;  // theta / 2pi in (-1/2, 1/2]
    const double sh = sinpi(x);
    const double s = sh * sh;                  // sin^2(theta/2)
    double sn, cs;
    sincospi(2.0 * x, &sn, &cs);               // sin theta, cos theta
    double rho, lg1p, arg;
    if (d.model == BINOMIAL) {
        const double wd = d.w0, wu = beta != 0.0 ? d.w1 * exp(beta) : d.w1;
        rho = wd + wu;
        lg1p = log1p(-4.0 * wd * wu * s / (rho * rho));
        arg = atan2(wu * sn, wd + wu * cs);
    } else {
        const double wm = beta != 0.0 ? d.w0 * exp(-beta) : d.w0, wc = d.w1;
        const double wp = beta != 0.0 ? d.w2 * exp(beta) : d.w2;
        rho = wm + wc + wp;
        const double sp = wp + wm, df = wp - wm;
        const double delta = (-4.0 * s * (rho * sp - df * df) + 16.0 * wp * wm * s * s) / (rho * rho);
        lg1p = log1p(delta);
        arg = atan2(df * sn, rho - 2.0 * sp * s);
    }
    const double lrel = 0.5 * (double)h * lg1p;  // log(|P|^h / rho^h)
    if (!(lrel > -60.0)) return make_double2(0.0, 0.0);
    const double mag = exp((double)h * log(rho) + lrel + lscale);
    double ps, pc;
    sincos((double)h * arg, &ps, &pc);
    return make_double2(mag * pc, mag * ps);
}

// ------------------------------------------------------ FFT correlation
__device__ __forceinline__ double tilt_in(double x, double beta, ll t, double tc)
{
    return (beta == 0.0 || x == 0.0) ? x : x * exp(-beta * ((double)t - tc));
}
__device__ __forceinline__ double tilt_out(double y, double beta, ll m)
{
    return beta == 0.0 ? y : y * exp(beta * (double)m);
}

// dst[t] = (x (*) W^(h))[out_off + t], t in [0, n_out), where x = src[0..n_in)
// zero-padded to N = 2^ceil(log2 n_in) and (*) is the circular correlation of
// the h-step kernel; for out_off + n_out <= n_in - span the window never wraps.
// Whole workgroup.  N <= 2048: in LDS.  Larger N: four-step with N = N1 * 2048
// through the global scratch `scr` (N complex).
// With beta != 0 the input is tilted, x~_t = x_t e^{-beta (t - tc)}, the kernel
// spectrum is tilted to match and the output is untilted, y_m = y~_m e^{beta m}
// (the e^{-beta tc} factor rides in the spectrum), so that a segment whose
// values grow like e^{beta t} is transformed at uniform relative precision.
__device__ void fft_correlate(const Desc &d, const double *__restrict__ src, ll n_in, ll h,
                              ll out_off, ll n_out, double *__restrict__ dst, double2 *scr,
                              double2 *lds, const double2 *__restrict__ tw, double beta = 0.0,
                              double tc = 0.0)
{
    if (n_out <= 0) return;
    const double lscale = -beta * tc;
    int lgN = ceil_log2(n_in);
    if (lgN < 1) lgN = 1;
    const ll N = ll(1) << lgN;
    const double invN = 1.0 / (double)N;
    const int tid = threadIdx.x;
    if (lgN <= LG_NLDS) {
        for (int t = tid; t < N; t += WG) lds[t] = make_double2(t < n_in ? tilt_in(src[t], beta, t, tc) : 0.0, 0.0);
        __syncthreads();
        lds_dif(lds, lgN, 1, tw);
        for (int t = tid; t < N; t += WG)
            lds[t] = cmul(lds[t], kernel_power(d, h, bitrev(t, lgN), lgN, beta, lscale));
        __syncthreads();
        lds_dit_inv(lds, lgN, 1, tw);
        for (ll t = tid; t < n_out; t += WG) dst[t] = tilt_out(lds[out_off + t].x * invN, beta, out_off + t);
        __syncthreads();
        return;
    }
    const int lg2 = LG_NLDS;
    const ll N2 = ll(1) << lg2;
    const int lg1 = lgN - lg2;
    const int N1 = 1 << lg1;
    const int C = NLDS >> lg1;  // columns per LDS tile
    const int twsh = LG_TW - lgN;
    // 1. column transforms (length N1) of the N1 x N2 row-major view, times
    //    the twiddle w_N^{n2 k1}; rows stay in bit-reversed k1 order.
    for (ll n20 = 0; n20 < N2; n20 += C) {
        for (int t = tid; t < NLDS; t += WG) {
            const int c = t % C, n1 = t / C;
            const ll idx = (ll)n1 * N2 + n20 + c;
            lds[c * N1 + n1] = make_double2(idx < n_in ? tilt_in(src[idx], beta, idx, tc) : 0.0, 0.0);
        }
        __syncthreads();
        lds_dif(lds, lg1, C, tw);
        for (int t = tid; t < NLDS; t += WG) {
            const int c = t % C, p1 = t / C;
            const ll k1 = bitrev(p1, lg1), n2 = n20 + c;
            const double2 w = tw[((n2 * k1) & (N - 1)) << twsh];
            scr[(ll)p1 * N2 + n2] = cmul(lds[c * N1 + p1], w);
        }
        __syncthreads();
    }
    // 2. per row: forward length-N2 transform, multiply by the kernel power
    //    at frequency k1 + N1 k2, inverse transform.
    for (int p1 = 0; p1 < N1; ++p1) {
        const ll k1 = bitrev(p1, lg1);
        double2 *row = scr + (ll)p1 * N2;
        for (int t = tid; t < N2; t += WG) lds[t] = row[t];
        __syncthreads();
        lds_dif(lds, lg2, 1, tw);
        for (int t = tid; t < N2; t += WG) {
            const ll k2 = bitrev(t, lg2);
            lds[t] = cmul(lds[t], kernel_power(d, h, k1 + (ll)N1 * k2, lgN, beta, lscale));
        }
        __syncthreads();
        lds_dit_inv(lds, lg2, 1, tw);
        for (int t = tid; t < N2; t += WG) row[t] = lds[t];
        __syncthreads();
    }
    // 3. inverse column transforms after the conjugate twiddle; keep the window.
    for (ll n20 = 0; n20 < N2; n20 += C) {
        for (int t = tid; t < NLDS; t += WG) {
            const int c = t % C, p1 = t / C;
            const ll k1 = bitrev(p1, lg1), n2 = n20 + c;
            const double2 w = tw[((n2 * k1) & (N - 1)) << twsh];
            lds[c * N1 + p1] = cmulc(scr[(ll)p1 * N2 + n2], w);
        }
        __syncthreads();
        lds_dit_inv(lds, lg1, C, tw);
        for (int t = tid; t < NLDS; t += WG) {
            const int c = t % C, n1 = t / C;
            const ll idx = (ll)n1 * N2 + n20 + c;
            if (idx >= out_off && idx < out_off + n_out)
                dst[idx - out_off] = tilt_out(lds[c * N1 + n1].x * invN, beta, idx);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void count_conv(Stats *st, ll n_in, ll n_out)
{
    if (threadIdx.x == 0 && st && n_out > 0) {
        int l = ceil_log2(n_in);
        st->convs += 1;
        st->conv_in += n_in;
        st->conv_out += n_out;
        st->fft_points += ll(1) << (l < 1 ? 1 : l);
    }
}

// ------------------------------------------------------------ band walkers
// Executed by the 64 lanes of wave 0.  Lane l holds one cell of the current
// row; the neighbour a row step needs comes from the next lane, and cells
// beyond the band are exercise cells evaluated in closed form.  Each row's
// last continuation cell is found with a ballot; the boundary is kept within
// one cell per row of the previous one (Corollary 2.6 / Theorem 4.2), which
// only overrides the ballot at ties within rounding.

// Binomial: rows i0-1 .. i0-h from row i0, whose red cells are [c0, b]
// (b - c0 + 1 <= BAND); columns >= c0 only.  Writes the red cells of row i0-h
// to dst, the boundary of each row to bnd (may be NULL); returns the last red
// column of row i0-h.  *v0 receives the final value of column c0.
__device__ ll band_bin(const Desc &d, ll i0, ll c0, ll h, ll b, const double *src, double *dst,
                       ll *bnd, double *v0)
{
    const int l = threadIdx.x & 63;
    const ll j = c0 + l;
    double g = (j <= b) ? src[j] : ((j <= i0) ? ex_bin(d, i0, j) : 0.0);
    ll bc = b;
    for (ll k = 1; k <= h; ++k) {
        const ll i = i0 - k;
        double gn = __shfl_down(g, 1, 64);
        if (l == 63) gn = ex_bin(d, i + 1, c0 + BAND);  // exercise cell beyond the band
        const double c = d.w0 * g + d.w1 * gn;
        const double e = ex_bin(d, i, j);
        const bool red = (j <= i) && red_of(c, e);
        g = red ? c : e;
        const unsigned long long m = __ballot(red);
        const ll last = m ? c0 + 63 - __clzll(m) : c0 - 1;
        ll bn = last < bc - 1 ? bc - 1 : (last > bc ? bc : last);
        if (bn > i) bn = i;
        if (bn < c0 - 1) bn = c0 - 1;
        bc = bn;
        if (bnd && l == 0) bnd[i] = bc;
    }
    if (j <= bc) dst[j] = g;
    if (v0 && l == 0) *v0 = g;
    return bc;
}

// Trinomial: as band_bin; row i has columns 0..2i and each cell reads j, j+1,
// j+2.  Below an all-red row the boundary drops by two (the row shrinks), so
// the one-cell clamp only applies when the previous row had an exercise cell.
__device__ ll band_tri(const Desc &d, ll i0, ll c0, ll h, ll b, const double *src, double *dst,
                       ll *bnd, double *v0)
{
    const int l = threadIdx.x & 63;
    const ll j = c0 + l;
    double g = (j <= b) ? src[j] : ((j <= 2 * i0) ? ex_tri(d, i0, j) : 0.0);
    ll bc = b;
    for (ll k = 1; k <= h; ++k) {
        const ll i = i0 - k;
        double g1 = __shfl_down(g, 1, 64);
        double g2 = __shfl_down(g, 2, 64);
        if (l == 63) {
            g1 = ex_tri(d, i + 1, c0 + BAND);
            g2 = ex_tri(d, i + 1, c0 + BAND + 1);
        } else if (l == 62) {
            g2 = ex_tri(d, i + 1, c0 + BAND);
        }
        const double c = d.w0 * g + d.w1 * g1 + d.w2 * g2;
        const double e = ex_tri(d, i, j);
        const bool red = (j <= 2 * i) && red_of(c, e);
        g = red ? c : e;
        const unsigned long long m = __ballot(red);
        const ll last = m ? c0 + 63 - __clzll(m) : c0 - 1;
        ll bn;
        if (bc >= 2 * (i + 1))
            bn = last;  // previous row entirely red
        else
            bn = last < bc - 1 ? bc - 1 : (last > bc ? bc : last);
        if (bn > 2 * i) bn = 2 * i;
        if (bn < c0 - 1) bn = c0 - 1;
        bc = bn;
        if (bnd && l == 0) bnd[i] = bc;
    }
    if (j <= bc) dst[j] = g;
    if (v0 && l == 0) *v0 = g;
    return bc;
}

// BSM put: steps n0+1 .. n0+h from step n0, whose exercise cells are k <= f
// and whose continuation cells [f+1, R0] are read from src (absolute k).  The
// band's right edge starts at R0 and moves left one cell per step (the
// dependency cone), its left part stays inside the exercise region (needs
// R0 - f <= 62).  Writes the red cells of step n0+h, up to R0-h, to dst and
// returns the last exercise offset of step n0+h.  *vr receives the value of
// the rightmost cell (the apex when R0 - h = 0).
__device__ ll band_bsm(const Desc &d, ll n0, ll f, ll h, ll R0, const double *src, double *dst,
                       ll *bnd, double *vr)
{
    const int l = threadIdx.x & 63;
    const ll T = d.T;
    ll base = R0 - 63;
    ll k = base + l;
    double v = (k <= f) ? ex_bsm(d, k) : src[k];
    ll fc = f;
    for (ll t = 1; t <= h; ++t) {
        base -= 1;
        k = base + l;
        // new cell k needs old cells k-1, k, k+1 = old lanes l-2, l-1, l
        double vm2 = __shfl_up(v, 2, 64);
        double vm1 = __shfl_up(v, 1, 64);
        if (l == 0) {
            vm2 = ex_bsm(d, k - 1);
            vm1 = ex_bsm(d, k);
        } else if (l == 1) {
            vm2 = ex_bsm(d, k - 1);
        }
        const double cont = d.w0 * vm2 + d.w1 * vm1 + d.w2 * v;
        const double g = ex_bsm(d, k);
        const bool green = g > cont;
        v = green ? g : cont;
        const unsigned long long m = __ballot(green);
        const ll last = m ? base + 63 - __clzll(m) : base - 1;
        ll fn = last < fc - 1 ? fc - 1 : (last > fc ? fc : last);
        fc = fn;
        if (bnd && l == 0) {
            const ll n = n0 + t;
            bnd[n] = (fc < -(T - n)) ? BSM_NONE : (fc > T - n ? T - n : fc);
        }
    }
    if (k > fc && k <= R0 - h) dst[k] = v;
    if (vr && l == 63) *vr = v;
    return fc;
}

// ---------------------------------------------------------- the recursion
struct Frame {
    ll r0;    // row i0 (lattices) / step n (BSM)
    ll c0;    // first red column (lattices) / boundary f (BSM)
    ll h;     // trapezoid height
    ll b;     // last red column of row r0 (lattices)
    ll aoff;  // arena offset (doubles) of this frame's middle-row buffer
    ll ret1;  // boundary returned by the first sub-trapezoid
    double *src, *dst, *mid;
    int stage, pad;
};

struct Ctx {
    const Desc *d;
    Stats *st;  // work counters in LDS (updated by lane 0 only)
    double *lo, *hi;  // this option's workspace (doubles) for range checks
    double *arena;
    ll arena_len;
    double2 *scr;
    double2 *lds;
    const double2 *tw;
    ll *bnd;
};

__device__ __forceinline__ bool in_ws(const Ctx &cx, const double *p, ll first, ll last)
{
    if (last < first) return true;
    return (p + first >= cx.lo) && (p + last < cx.hi);
}

// Solve one trapezoid (model-dependent geometry, see the frame stages below)
// and return the boundary of its last row.  All lanes call it; control flow is
// uniform.  On a failed range check the error is stored in *err.
__device__ ll solve_trapezoid(const Ctx &cx, Frame root, Frame *stk, int *sp_sh, ll *ret_sh,
                              int *err_sh, ll *leaf_sh)
{
    const Desc &d = *cx.d;
    const int tid = threadIdx.x;
    const int span = (d.model == BINOMIAL) ? 1 : 2;  // columns consumed per row (lattices)
    if (tid == 0) {
        stk[0] = root;
        *sp_sh = 0;
    }
    __syncthreads();
    for (;;) {
        const int s = *sp_sh;
        if (s < 0 || *err_sh) break;
        Frame fr = stk[s];
        const ll rv = *ret_sh;
        __syncthreads();
        bool pop = false;
        ll result = 0;
        Frame child;
        int e = DEV_OK;
        if (d.model != BSM) {
            // Lattice trapezoid (i0 = r0): red cells [c0, b] of row i0 in src;
            // produces the red cells of row i0 - h in dst.
            const ll i0 = fr.r0, c0 = fr.c0, h = fr.h, b = fr.b;
            const ll h1 = h / 2, h2 = h - h1;
            const ll nred = b - c0 + 1;
            if (fr.stage == 0) {
                if (nred <= BAND) {
                    if (!in_ws(cx, fr.src, c0, b) || !in_ws(cx, fr.dst, c0, c0 + BAND - 1)) {
                        e = DEV_RANGE;
                    } else {
                        if (tid < 64) {
                            const ll r = (d.model == BINOMIAL)
                                             ? band_bin(d, i0, c0, h, b, fr.src, fr.dst, cx.bnd, nullptr)
                                             : band_tri(d, i0, c0, h, b, fr.src, fr.dst, cx.bnd, nullptr);
                            if (tid == 0) {
                                *leaf_sh = r;
                                cx.st->band_rows += h;
                            }
                        }
                        __syncthreads();
                        result = *leaf_sh;
                    }
                    pop = true;
                } else {
                    // (1) row r = i0 - h1, columns [c0, b - span h1], by FFT from row i0.
                    double *mid = cx.arena + fr.aoff - c0;
                    if (fr.aoff + nred > cx.arena_len) e = DEV_ARENA;
                    else if (!in_ws(cx, fr.src, c0, b)) e = DEV_RANGE;
                    else {
                        count_conv(cx.st, nred, nred - span * h1);
                        fft_correlate(d, fr.src + c0, nred, h1, (span == 1) ? 0 : h1, nred - span * h1,
                                      mid + c0, cx.scr, cx.lds, cx.tw);
                        fr.mid = mid;
                        fr.stage = 1;
                        // (2) sub-trapezoid on the last span*h1 red cells of row i0
                        child = Frame{i0, b - span * h1 + 1, h1, b, fr.aoff + nred, 0, fr.src, mid, nullptr, 0, 0};
                    }
                }
            } else if (fr.stage == 1) {
                // (3) row i0 - h, columns [c0, br - span h2], by FFT from row r.
                const ll br = rv;
                const ll n2 = br - c0 + 1;
                if (!in_ws(cx, fr.mid, c0, br) || !in_ws(cx, fr.dst, c0, br)) e = DEV_RANGE;
                else {
                    count_conv(cx.st, n2, n2 - span * h2);
                    if (n2 - span * h2 > 0)
                        fft_correlate(d, fr.mid + c0, n2, h2, (span == 1) ? 0 : h2, n2 - span * h2,
                                      fr.dst + c0, cx.scr, cx.lds, cx.tw);
                    fr.ret1 = br;
                    fr.stage = 2;
                    // (4) sub-trapezoid on the last span*h2 red cells of row r
                    child = Frame{i0 - h1, br - span * h2 + 1, h2, br, fr.aoff + nred, 0, fr.mid, fr.dst,
                                  nullptr, 0, 0};
                }
            } else {
                result = rv;
                pop = true;
            }
        } else {
            // BSM trapezoid centred on the boundary f = c0 of step n = r0: the
            // red cells [f+1, f+2h] of step n in src produce step n+h on
            // [f-h, f+h] (red part) in dst.
            const ll n = fr.r0, f = fr.c0, h = fr.h;
            const ll h1 = h / 2, h2 = h - h1;
            if (fr.stage == 0) {
                if (h <= (BAND - 2) / 2) {
                    if (!in_ws(cx, fr.src, f + 1, f + 2 * h) || !in_ws(cx, fr.dst, f - h, f + h)) {
                        e = DEV_RANGE;
                    } else {
                        if (tid < 64) {
                            const ll r = band_bsm(d, n, f, h, f + 2 * h, fr.src, fr.dst, cx.bnd, nullptr);
                            if (tid == 0) {
                                *leaf_sh = r;
                                cx.st->band_rows += h;
                            }
                        }
                        __syncthreads();
                        result = *leaf_sh;
                    }
                    pop = true;
                } else {
                    // middle step n+h1 on [f-h1+1, f+h+h2] (2h cells)
                    const ll base = f - h1 + 1;
                    double *mid = cx.arena + fr.aoff - base;
                    if (fr.aoff + 2 * h > cx.arena_len) e = DEV_ARENA;
                    else if (!in_ws(cx, fr.src, f + 1, f + 2 * h)) e = DEV_RANGE;
                    else {
                        // conv 1: red cells [f+1, f+2h] -> [f+1+h1, f+2h-h1] of step n+h1
                        count_conv(cx.st, 2 * h, 2 * h - 2 * h1);
                        fft_correlate(d, fr.src + f + 1, 2 * h, h1, h1, 2 * h - 2 * h1, mid + f + 1 + h1,
                                      cx.scr, cx.lds, cx.tw);
                        fr.mid = mid;
                        fr.stage = 1;
                        child = Frame{n, f, h1, 0, fr.aoff + 2 * h, 0, fr.src, mid, nullptr, 0, 0};
                    }
                }
            } else if (fr.stage == 1) {
                const ll fp = rv;  // boundary of step n+h1, in [f-h1, f]
                const ll nin = f + h + h2 - fp;
                if (fp < f - h1 || fp > f) e = DEV_RANGE;
                else if (!in_ws(cx, fr.mid, fp + 1, f + h + h2) || !in_ws(cx, fr.dst, fp + 1 + h2, f + h)) e = DEV_RANGE;
                else {
                    // conv 2: red cells [f'+1, f+h+h2] of step n+h1 -> [f'+1+h2, f+h] of step n+h
                    count_conv(cx.st, nin, nin - 2 * h2);
                    fft_correlate(d, fr.mid + fp + 1, nin, h2, h2, nin - 2 * h2, fr.dst + fp + 1 + h2,
                                  cx.scr, cx.lds, cx.tw);
                    fr.ret1 = fp;
                    fr.stage = 2;
                    child = Frame{n + h1, fp, h2, 0, fr.aoff + 2 * h, 0, fr.mid, fr.dst, nullptr, 0, 0};
                }
            } else {
                result = rv;
                pop = true;
            }
        }
        if (tid == 0) {
            if (e != DEV_OK) {
                *err_sh = e;
            } else if (pop) {
                *ret_sh = result;
                *sp_sh = s - 1;
            } else if (s + 1 >= MAXD) {
                *err_sh = DEV_STACK;
            } else {
                stk[s] = fr;
                stk[s + 1] = child;
                *sp_sh = s + 1;
                if (s + 1 > cx.st->max_depth) cx.st->max_depth = s + 1;
            }
        }
        __syncthreads();
    }
    const ll r = *ret_sh;
    __syncthreads();
    return r;
}

// --------------------------------------------------------------- drivers
__device__ double drive_lattice(const Ctx &cx, double *rowA, double *rowB, Frame *stk, int *sp_sh,
                                ll *ret_sh, int *err_sh, ll *leaf_sh, ll *red_sh, double *val_sh)
{
    const Desc &d = *cx.d;
    const ll T = d.T;
    const int tid = threadIdx.x;
    const bool bin = d.model == BINOMIAL;
    const ll wT = bin ? T : 2 * T;  // last column of row T
    // Expiry row T (red = out of the money: G^red = 0 >= G^green) and row T-1.
    ll lastT = -1, lastT1 = -1;
    for (ll j = tid; j <= wT; j += WG) {
        const double eT = bin ? ex_bin(d, T, j) : ex_tri(d, T, j);
        if (red_of(0.0, eT)) lastT = j;
        if (j <= wT - (bin ? 1 : 2)) {
            double c;
            if (bin) {
                const double e1 = ex_bin(d, T, j + 1);
                const double g0 = red_of(0.0, eT) ? 0.0 : eT, g1 = red_of(0.0, e1) ? 0.0 : e1;
                c = d.w0 * g0 + d.w1 * g1;
            } else {
                const double e1 = ex_tri(d, T, j + 1), e2 = ex_tri(d, T, j + 2);
                const double g0 = red_of(0.0, eT) ? 0.0 : eT, g1 = red_of(0.0, e1) ? 0.0 : e1,
                             g2 = red_of(0.0, e2) ? 0.0 : e2;
                c = d.w0 * g0 + d.w1 * g1 + d.w2 * g2;
            }
            const double e = bin ? ex_bin(d, T - 1, j) : ex_tri(d, T - 1, j);
            const bool red = red_of(c, e);
            rowA[j] = red ? c : e;
            if (red) lastT1 = j;
        }
    }
    if (tid == 0) cx.st->direct_cells += wT + 1 - (bin ? 1 : 2);
    lastT = block_max(lastT, red_sh);
    lastT1 = block_max(lastT1, red_sh);
    if (cx.bnd && tid == 0) {
        cx.bnd[T] = lastT;
        cx.bnd[T - 1] = lastT1;
    }
    ll i0 = T - 1, b = lastT1;
    double *src = rowA, *dst = rowB;
    if (T > 1 && (d.no_green || b == wT - (bin ? 1 : 2))) {
        // No exercise cell below the expiry row: with Y = 0 Lemma 2.3 leaves
        // none (the classification of far in-the-money cells of row T-1 is
        // then rounding noise), and an entirely red row T-1 keeps every row
        // below red (Corollary 2.6: the boundary drops at most one cell per
        // row while the row shrinks by one or two).  The root is then one
        // linear functional of row T-1, whose values grow like S u^{col}, so
        // the correlation is tilted about the at-the-money column tc.
        b = wT - (bin ? 1 : 2);
        if (cx.bnd && tid == 0) cx.bnd[T - 1] = b;
        const double beta = bin ? 2.0 * d.a : d.a;
        double tc = bin ? 0.5 * ((double)(T - 1) + log(d.K / d.S) / d.a)
                        : (double)(T - 1) + log(d.K / d.S) / d.a;
        if (tc < 0.0) tc = 0.0;
        if (tc > (double)b) tc = (double)b;
        if (cx.bnd)
            for (ll i = tid; i < T - 1; i += WG) cx.bnd[i] = bin ? i : 2 * i;
        const ll hh = T - 1;
        count_conv(cx.st, b + 1, 1);
        fft_correlate(d, src, b + 1, hh, bin ? 0 : hh, 1, val_sh, cx.scr, cx.lds, cx.tw, beta, tc);
        __syncthreads();
        return *val_sh;
    }
    while (i0 > 0) {
        if (b < 0) {  // no red cell: every row below is green (Lemma 2.4)
            if (cx.bnd)
                for (ll i = tid; i < i0; i += WG) cx.bnd[i] = -1;
            __syncthreads();
            return d.S - d.K;
        }
        const ll nred = b + 1;
        if (nred <= BAND) {  // the band walks the leftover triangle to the root
            if (tid == 0) cx.st->band_rows += i0;
            if (tid < 64) {
                if (bin) band_bin(d, i0, 0, i0, b, src, dst, cx.bnd, val_sh);
                else band_tri(d, i0, 0, i0, b, src, dst, cx.bnd, val_sh);
            }
            __syncthreads();
            return *val_sh;
        }
        ll h = bin ? nred : nred / 2;
        if (h > i0) h = i0;
        Frame root{i0, 0, h, b, 0, 0, src, dst, nullptr, 0, 0};
        if (tid == 0) cx.st->trapezoids += 1;
        b = solve_trapezoid(cx, root, stk, sp_sh, ret_sh, err_sh, leaf_sh);
        if (*err_sh) return NAN;
        i0 -= h;
        double *t = src;
        src = dst;
        dst = t;
    }
    const double p = (b >= 0) ? src[0] : d.S - d.K;
    __syncthreads();
    return p;
}

__device__ double drive_bsm(const Ctx &cx, double *rowA, double *rowB, Frame *stk, int *sp_sh,
                            ll *ret_sh, int *err_sh, ll *leaf_sh, ll *red_sh, double *val_sh)
{
    const Desc &d = *cx.d;
    const ll T = d.T;
    const int tid = threadIdx.x;
    const ll NONE = LLONG_MIN;
    // rows are indexed by k in [-2T-1, T+1] -> pointer offset 2T+1
    double *A = rowA + 2 * T + 1, *B = rowB + 2 * T + 1;
    ll f0 = NONE, f1 = NONE;
    for (ll k = -T + tid; k <= T; k += WG) {
        const double g = ex_bsm(d, k);
        if (g > 0.0) f0 = k;
        if (k >= -(T - 1) && k <= T - 1) {
            const double gm = ex_bsm(d, k - 1), gp = ex_bsm(d, k + 1);
            const double cont = d.w0 * (gm > 0.0 ? gm : 0.0) + d.w1 * (g > 0.0 ? g : 0.0) +
                                 d.w2 * (gp > 0.0 ? gp : 0.0);
            const bool green = g > cont;
            A[k] = green ? g : cont;
            if (green) f1 = k;
        }
    }
    if (tid == 0) cx.st->direct_cells += 2 * T - 1;
    f0 = block_max(f0, red_sh);
    f1 = block_max(f1, red_sh);
    if (cx.bnd && tid == 0) {
        cx.bnd[0] = f0;
        cx.bnd[1] = (T >= 1) ? f1 : NONE;
    }
    ll n = 1, R = T - 1, L = -(T - 1);
    ll f = (f1 == NONE) ? L - 1 : f1;
    double *src = A, *dst = B;
    for (;;) {
        if (n == T) {
            const double v = (f >= 0) ? ex_bsm(d, 0) : src[0];
            __syncthreads();
            return d.K * v;
        }
        if (f < L) {  // no exercise cell left in the cone: the rest is linear
            if (cx.bnd)
                for (ll m = n + 1 + tid; m <= T; m += WG) cx.bnd[m] = NONE;
            const ll hh = T - n;
            count_conv(cx.st, R - L + 1, 1);
            fft_correlate(d, src + L, R - L + 1, hh, hh, 1, val_sh, cx.scr, cx.lds, cx.tw);
            __syncthreads();
            return d.K * (*val_sh);
        }
        if (f >= R) {  // the whole cone exercises, and keeps doing so
            if (cx.bnd)
                for (ll m = n + 1 + tid; m <= T; m += WG) cx.bnd[m] = T - m;
            __syncthreads();
            return d.K * ex_bsm(d, 0);
        }
        const ll w = R - f;
        if (w <= BAND - 2) {  // the band walks the leftover cone to the apex
            if (tid == 0) cx.st->band_rows += T - n;
            if (tid < 64) band_bsm(d, n, f, T - n, R, src, dst, cx.bnd, val_sh);
            __syncthreads();
            return d.K * (*val_sh);
        }
        ll h = w / 2;
        if (h > T - n) h = T - n;
        Frame root{n, f, h, 0, 0, 0, src, dst, nullptr, 0, 0};
        if (tid == 0) cx.st->trapezoids += 1;
        const ll fn = solve_trapezoid(cx, root, stk, sp_sh, ret_sh, err_sh, leaf_sh);
        if (*err_sh) return NAN;
        // the rest of step n+h: red cells [f+1+h, R-h] from [f+1, R] of step n
        count_conv(cx.st, w, w - 2 * h);
        fft_correlate(d, src + f + 1, w, h, h, w - 2 * h, dst + f + 1 + h, cx.scr, cx.lds, cx.tw);
        n += h;
        R -= h;
        L += h;
        f = fn;
        double *t = src;
        src = dst;
        dst = t;
    }
}

__global__ void __launch_bounds__(WG) solve_kernel(const Desc *__restrict__ descs, char *ws,
                                                   const double2 *__restrict__ tw, double *price,
                                                   ll *bnd, ll bnd_stride, int32_t *err, Stats *stats)
{
    __shared__ double2 lds[NLDS];
    __shared__ Frame stk[MAXD];
    __shared__ int sp_sh, err_sh;
    __shared__ ll ret_sh, leaf_sh, red_sh[WG / 64];
    __shared__ double val_sh;
    __shared__ Stats st_sh;

    const Desc d = descs[blockIdx.x];
    if (d.model < 0) {  // rejected on the host: no work, price NaN
        if (threadIdx.x == 0) {
            price[d.out_index] = NAN;
            stats[d.out_index] = Stats{0, 0, 0, 0, 0, 0, 0, 0};
        }
        return;
    }
    char *base = ws + d.ws_off;
    double *rowA = (double *)base;
    double *rowB = rowA + d.row_len;
    double *arena = rowB + d.row_len;
    double2 *scr = (double2 *)(arena + d.arena_len);
    Ctx cx;
    cx.d = &d;
    cx.lo = rowA;
    cx.hi = (double *)(scr + d.nfft);
    cx.arena = arena;
    cx.arena_len = d.arena_len;
    cx.scr = scr;
    cx.lds = lds;
    cx.tw = tw;
    cx.bnd = bnd ? bnd + d.out_index * bnd_stride : nullptr;
    cx.st = &st_sh;
    if (threadIdx.x == 0) {
        err_sh = 0;
        ret_sh = 0;
        st_sh = Stats{0, 0, 0, 0, 0, 0, 0, 0};
    }
    __syncthreads();
    double p;
    if (d.model == BSM)
        p = drive_bsm(cx, rowA, rowB, stk, &sp_sh, &ret_sh, &err_sh, &leaf_sh, red_sh, &val_sh);
    else
        p = drive_lattice(cx, rowA, rowB, stk, &sp_sh, &ret_sh, &err_sh, &leaf_sh, red_sh, &val_sh);
    __syncthreads();
    if (threadIdx.x == 0) {
        price[d.out_index] = err_sh ? NAN : p;
        if (err) err[d.out_index] = err_sh;
        stats[d.out_index] = st_sh;
    }
}

__global__ void twiddle_kernel(double2 *tw)
{
    const ll t = (ll)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < TW_N) {
        double s, c;
        sincospi(2.0 * (double)t / (double)TW_N, &s, &c);
        tw[t] = make_double2(c, -s);  // e^{-2 pi i t / TW_N}
    }
}

int launch_twiddles(void *d_tw, void *stream)
{
    hipLaunchKernelGGL(twiddle_kernel, dim3((unsigned)(TW_N / 256)), dim3(256), 0, (hipStream_t)stream,
                       (double2 *)d_tw);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

int launch_solve(const Desc *d_desc, int64_t n, char *d_ws, const void *d_tw, double *d_price,
                 int64_t *d_bnd, int64_t bnd_stride, int32_t *d_err, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(solve_kernel, dim3((unsigned)n), dim3(WG), 0, (hipStream_t)stream, d_desc, d_ws,
                       (const double2 *)d_tw, d_price, (ll *)d_bnd, (ll)bnd_stride, d_err,
                       (Stats *)(d_ws + stats_offset(n)));
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

}  // namespace aop
