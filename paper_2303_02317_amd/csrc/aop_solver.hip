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

// Model parameters, passed by value so that they live in registers.
struct Mp {
    int model;
    ll T, no_green;
    double S, K, a, s0, w0, w1, w2;
};
__device__ __forceinline__ Mp make_mp(const Desc &d)
{
    Mp p;
    p.model = d.model;
    p.T = d.T;
    p.no_green = d.no_green;
    p.S = d.S;
    p.K = d.K;
    p.a = d.a;
    p.s0 = d.s0;
    p.w0 = d.w0;
    p.w1 = d.w1;
    p.w2 = d.w2;
    return p;
}

// Wave-uniform copy of a value that is uniform by construction.
__device__ __forceinline__ ll uni(ll v)
{
    const int lo = __builtin_amdgcn_readfirstlane((int)(unsigned)(v & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return (ll)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
// DPP wave shifts (gfx9 wave_shl1 / wave_shr1): value of lane l+1 (lane 63
// receives `fill`), value of lane l-1 (lane 0 receives `fill`).  All 64 lanes
// must be active.
__device__ __forceinline__ double dpp_dn1(double v, double fill)
{
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(fill), __double2loint(v), 0x130, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(fill), __double2hiint(v), 0x130, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double dpp_up1(double v, double fill)
{
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(fill), __double2loint(v), 0x138, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(fill), __double2hiint(v), 0x138, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

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
__device__ __forceinline__ double ex_bin(const Mp &d, ll i, ll j)
{
    return d.S * exp((double)(2 * j - i) * d.a) - d.K;  // S u^{2j-i} - K
}
__device__ __forceinline__ double ex_tri(const Mp &d, ll i, ll j)
{
    return d.S * exp((double)(j - i) * d.a) - d.K;  // S u^{j-i} - K
}
__device__ __forceinline__ double ex_bsm(const Mp &d, ll k)
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

// ------------------------------------------------------------ LDS FFT
// nb batched transforms of length 2^lg <= 2048, stored contiguously in LDS.
// Forward: decimation in frequency, natural order in -> bit-reversed out.
// Inverse (unnormalised): decimation in time, bit-reversed in -> natural out.
// Each pass loads 2^K elements per lane, applies K radix-2 stages in
// registers and stores them back, so a 2048-point transform takes four LDS
// round trips.  twl holds e^{-2 pi i t / 2048}, t < 1024.
template <int K, bool INV>
__device__ __forceinline__ void lds_pass(double2 *x, int lg, int nb, int s_lo, const double2 *twl)
{
    constexpr int G = 1 << K;
    const int n = 1 << lg;
    const int s_hi = s_lo + K - 1;
    const int per = n >> K;  // groups per transform
    const int groups = nb * per;
    const int jmask = (1 << s_lo) - 1;
    for (int gi = threadIdx.x; gi < groups; gi += WG) {
        const int b = gi / per;
        const int r = gi - b * per;
        const int j = r & jmask;
        const int blk = r >> s_lo;
        const int base = b * n + (blk << (s_hi + 1)) + j;
        double2 v[G];
#pragma unroll
        for (int q = 0; q < G; ++q) v[q] = x[base + (q << s_lo)];
        if (!INV) {
#pragma unroll
            for (int t = K - 1; t >= 0; --t) {
                const int s = s_lo + t;
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    if (q & (1 << t)) continue;
                    const int jj = ((q & ((1 << t) - 1)) << s_lo) + j;
                    const double2 w = twl[jj << (10 - s)];
                    const double2 u = v[q], z = v[q + (1 << t)];
                    v[q] = make_double2(u.x + z.x, u.y + z.y);
                    v[q + (1 << t)] = cmul(make_double2(u.x - z.x, u.y - z.y), w);
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < K; ++t) {
                const int s = s_lo + t;
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    if (q & (1 << t)) continue;
                    const int jj = ((q & ((1 << t) - 1)) << s_lo) + j;
                    const double2 w = twl[jj << (10 - s)];
                    const double2 u = v[q], z = cmulc(v[q + (1 << t)], w);
                    v[q] = make_double2(u.x + z.x, u.y + z.y);
                    v[q + (1 << t)] = make_double2(u.x - z.x, u.y - z.y);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < G; ++q) x[base + (q << s_lo)] = v[q];
    }
    __syncthreads();
}

__device__ void lds_dif(double2 *x, int lg, int nb, const double2 *twl)
{
    int s_hi = lg - 1;
    while (s_hi >= 0) {
        const int k = s_hi + 1 >= 3 ? 3 : s_hi + 1;
        const int s_lo = s_hi - k + 1;
        if (k == 3) lds_pass<3, false>(x, lg, nb, s_lo, twl);
        else if (k == 2) lds_pass<2, false>(x, lg, nb, s_lo, twl);
        else lds_pass<1, false>(x, lg, nb, s_lo, twl);
        s_hi = s_lo - 1;
    }
}

__device__ void lds_dit_inv(double2 *x, int lg, int nb, const double2 *twl)
{
    int s_lo = 0;
    while (s_lo < lg) {
        const int k = lg - s_lo >= 3 ? 3 : lg - s_lo;
        if (k == 3) lds_pass<3, true>(x, lg, nb, s_lo, twl);
        else if (k == 2) lds_pass<2, true>(x, lg, nb, s_lo, twl);
        else lds_pass<1, true>(x, lg, nb, s_lo, twl);
        s_lo += k;
    }
}

// ------------------------------------------------- h-step kernel spectrum
// Correlation y_m = sum_t W_t x_{m+t} with the h-fold one-step stencil has
// DFT multiplier P(theta)^h, P(theta) = sum_t w_t e^{i t theta}.  Evaluated in
// polar form in FP64: |P|^2 = rho^2 (1 + delta) with delta computed from
// s = sin^2(theta/2) without cancellation, log1p for the magnitude and atan2
// for the phase, so the h-th power costs O(1) and its relative error does not
// grow with h (repeated squaring would lose h ulps).
//   binomial:  P = w_dn + w_up e^{i theta}                  (one-sided, offsets 0, 1)
//   trinomial / BSM: P = w_m e^{-i theta} + w_c + w_p e^{i theta}  (centred)
// An exponential tilt beta (used only where a red segment spans a huge
// dynamic range) replaces w_t by w_t e^{beta t} and adds lscale to the
// log-magnitude.  cos/sin of theta and sin(theta/2) come from the twiddle
// table.
struct Spec {
    int bin;
    double h, wa, wb, wc;  // binomial: (w_dn, w_up); centred: (w_m, w_c, w_p)
    double rho, inv_rho2, lmag0, sp, df, cut;
};

__device__ __forceinline__ Spec make_spec(const Mp &p, ll h, double beta, double lscale)
{
    Spec q;
    q.bin = p.model == BINOMIAL;
    q.h = (double)h;
    if (q.bin) {
        q.wa = p.w0;
        q.wb = beta != 0.0 ? p.w1 * exp(beta) : p.w1;
        q.wc = 0.0;
        q.rho = q.wa + q.wb;
        q.sp = 0.0;
        q.df = 0.0;
    } else {
        q.wa = beta != 0.0 ? p.w0 * exp(-beta) : p.w0;
        q.wb = p.w1;
        q.wc = beta != 0.0 ? p.w2 * exp(beta) : p.w2;
        q.rho = q.wa + q.wb + q.wc;
        q.sp = q.wc + q.wa;
        q.df = q.wc - q.wa;
    }
    q.inv_rho2 = 1.0 / (q.rho * q.rho);
    q.lmag0 = q.h * log(q.rho) + lscale;
    q.cut = -120.0 / q.h;  // h delta / 2 < -60: below e^-60 of the kernel mass
    return q;
}

__device__ __forceinline__ double2 kernel_power(const Spec &q, ll f, int lgN, const double2 *__restrict__ tw)
{
    const double2 e = tw[f << (LG_TW - lgN)];  // e^{-i theta}, theta = 2 pi f / N
    const double cs = e.x, sn = -e.y;
    double sh;
    if (lgN < LG_TW) sh = tw[f << (LG_TW - 1 - lgN)].y;  // -sin(theta/2)
    else sh = sinpi((double)f / (double)(ll(1) << lgN));
    const double s = sh * sh;  // sin^2(theta/2)
    double delta, arg;
    if (q.bin) {
        delta = -4.0 * q.wa * q.wb * s * q.inv_rho2;
        if (delta < q.cut) return make_double2(0.0, 0.0);
        arg = atan2(q.wb * sn, q.wa + q.wb * cs);
    } else {
        delta = (-4.0 * s * (q.rho * q.sp - q.df * q.df) + 16.0 * q.wc * q.wa * s * s) * q.inv_rho2;
        if (delta < q.cut) return make_double2(0.0, 0.0);
        arg = atan2(q.df * sn, q.rho - 2.0 * q.sp * s);
    }
    const double lrel = 0.5 * q.h * log1p(delta);
    if (!(lrel > -60.0)) return make_double2(0.0, 0.0);
    const double mag = exp(q.lmag0 + lrel);
    double ps, pc;
    sincos(q.h * arg, &ps, &pc);
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
__device__ __forceinline__ void fft_correlate(Mp p, const double *__restrict__ src, ll n_in_, ll h_,
                                           ll out_off_, ll n_out_, double *__restrict__ dst, double2 *scr,
                                           double2 *lds, const double2 *__restrict__ tw, const double2 *twl,
                                           double beta, double tc)
{
    const ll n_in = uni(n_in_), h = uni(h_), out_off = uni(out_off_), n_out = uni(n_out_);
    if (n_out <= 0) return;
    const Spec q = make_spec(p, h, beta, -beta * tc);
    int lgN = ceil_log2(n_in);
    if (lgN < 1) lgN = 1;
    const ll N = ll(1) << lgN;
    const double invN = 1.0 / (double)N;
    const int tid = threadIdx.x;
    if (lgN <= LG_NLDS) {
        for (int t = tid; t < N; t += WG) lds[t] = make_double2(t < n_in ? tilt_in(src[t], beta, t, tc) : 0.0, 0.0);
        __syncthreads();
        lds_dif(lds, lgN, 1, twl);
        // P(-theta) = conj(P(theta)): evaluate f <= N/2 and apply to both mirrors.
        for (ll f = tid; f <= N / 2; f += WG) {
            const double2 m = kernel_power(q, f, lgN, tw);
            const unsigned t1 = bitrev((unsigned)f, lgN), t2 = bitrev((unsigned)((N - f) & (N - 1)), lgN);
            lds[t1] = cmul(lds[t1], m);
            if (t2 != t1) lds[t2] = cmulc(lds[t2], m);
        }
        __syncthreads();
        lds_dit_inv(lds, lgN, 1, twl);
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
        lds_dif(lds, lg1, C, twl);
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
        lds_dif(lds, lg2, 1, twl);
        for (int t = tid; t < N2; t += WG) {
            const ll k2 = bitrev(t, lg2);
            lds[t] = cmul(lds[t], kernel_power(q, k1 + (ll)N1 * k2, lgN, tw));
        }
        __syncthreads();
        lds_dit_inv(lds, lg2, 1, twl);
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
        lds_dit_inv(lds, lg1, C, twl);
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

// ------------------------------------------------ direct correlation
// For short steps the h-step correlation is evaluated as h applications of
// the one-step linear stencil -- the backward recurrence itself without the
// max, valid because every cell involved is a continuation cell.  One wave
// holds the segment in registers (C cells per lane) and exchanges the edge
// cells with wave shuffles.  Lattices: dst[t] = y_t (one-sided form); BSM:
// dst[t] = z_{out_off + t} (centred form, out_off = h).
template <int C>
__device__ __forceinline__ void direct_wave(Mp p, const double *__restrict__ src, ll n_in_, ll h_, ll out_off_,
                                         ll n_out_, double *__restrict__ dst)
{
    const ll n_in = uni(n_in_), h = uni(h_), out_off = uni(out_off_), n_out = uni(n_out_);
    const int l = threadIdx.x & 63;
    double v[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const ll idx = (ll)l * C + c;
        v[c] = idx < n_in ? src[idx] : 0.0;
    }
    const double w0 = p.w0, w1 = p.w1, w2 = p.w2;
    if (p.model == BINOMIAL) {
        for (ll k = 0; k < h; ++k) {
            const double nb = dpp_dn1(v[0], 0.0);
#pragma unroll
            for (int c = 0; c < C - 1; ++c) v[c] = w0 * v[c] + w1 * v[c + 1];
            v[C - 1] = w0 * v[C - 1] + w1 * nb;
        }
    } else if (p.model == TRINOMIAL) {
        for (ll k = 0; k < h; ++k) {
            const double n0 = dpp_dn1(v[0], 0.0), n1 = dpp_dn1(v[1], 0.0);
#pragma unroll
            for (int c = 0; c < C - 2; ++c) v[c] = w0 * v[c] + w1 * v[c + 1] + w2 * v[c + 2];
            v[C - 2] = w0 * v[C - 2] + w1 * v[C - 1] + w2 * n0;
            v[C - 1] = w0 * v[C - 1] + w1 * n0 + w2 * n1;
        }
    } else {
        for (ll k = 0; k < h; ++k) {
            const double pv = dpp_up1(v[C - 1], 0.0), nv = dpp_dn1(v[0], 0.0);
            double prev = pv;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const double cur = v[c];
                const double nxt = (c + 1 < C) ? v[c + 1] : nv;
                v[c] = w0 * prev + w1 * cur + w2 * nxt;
                prev = cur;
            }
        }
    }
    const ll off = (p.model == BSM) ? out_off : 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const ll idx = (ll)l * C + c - off;
        if (idx >= 0 && idx < n_out) dst[idx] = v[c];
    }
}

#define DIRECT_MAX_H 160   // longest step count evaluated by direct stepping
#define DIRECT_MAX_N 1024  // longest segment (64 lanes x 16 cells)

__device__ __forceinline__ ll clk() { return (ll)__builtin_amdgcn_s_memtime(); }

// Dispatch: direct stepping for short kernels, FFT correlation otherwise.
__device__ __forceinline__ void correlate(Stats *st, const Mp &p, const double *__restrict__ src, ll n_in, ll h,
                                          ll out_off, ll n_out, double *__restrict__ dst, double2 *scr,
                                          double2 *lds, const double2 *__restrict__ tw, const double2 *twl,
                                          double beta = 0.0, double tc = 0.0)
{
    if (n_out <= 0) return;
    const ll t0 = clk();
    if (beta == 0.0 && h <= DIRECT_MAX_H && n_in <= DIRECT_MAX_N) {
        if (threadIdx.x < 64) {
            if (n_in <= 128) direct_wave<2>(p, src, n_in, h, out_off, n_out, dst);
            else if (n_in <= 256) direct_wave<4>(p, src, n_in, h, out_off, n_out, dst);
            else if (n_in <= 512) direct_wave<8>(p, src, n_in, h, out_off, n_out, dst);
            else direct_wave<16>(p, src, n_in, h, out_off, n_out, dst);
        }
        __syncthreads();
        if (threadIdx.x == 0 && st) {
            st->n_direct += 1;
            st->cyc_direct += clk() - t0;
        }
        return;
    }
    fft_correlate(p, src, n_in, h, out_off, n_out, dst, scr, lds, tw, twl, beta, tc);
    if (threadIdx.x == 0 && st) {
        st->n_fft += 1;
        st->cyc_fft += clk() - t0;
    }
}

// ------------------------------------------------------------ band walkers
// Executed by the 64 lanes of wave 0.  Lane l holds one cell of the current
// row; the neighbour a row step needs comes from the next lane by a DPP wave
// shift, and the cell beyond the band (an exercise cell) rides in as the
// shift's fill value.  Exercise values are carried per lane by one
// multiplication per row (S u^{col-i} gains a factor u per row down) and
// re-seeded with exp() every RESEED rows.
//
// Boundary tracking uses the structure the paper proves: from one row to the
// next the last continuation cell either stays or moves one cell towards the
// root's side (Corollary 2.6, Theorem 4.2).  So each row only tests the ballot
// bit of the previous boundary cell: set -> the boundary stays, clear -> it
// drops by one.  This is the rule the oracle's last-red scan follows wherever
// the red cells are contiguous; the two can differ only where rounding makes a
// near-tie cell flip.  Per-row boundaries are collected (one row per lane, 64
// rows per store) only when the caller asks for them.
#define RESEED 64

__device__ __forceinline__ unsigned long long row_mask(int last_lane)  // lanes 0..last_lane
{
    if (last_lane < 0) return 0ull;
    if (last_lane >= 63) return ~0ull;
    return (1ull << (last_lane + 1)) - 1ull;
}

__device__ __forceinline__ double vmax_f64(double a, double b)
{
    double r;
    asm volatile("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;  // IEEE maxNum: a NaN operand yields the other one
}

// Lane `lane` of the result takes the (uniform) value `val`; other lanes keep `dst`.
__device__ __forceinline__ unsigned writelane(unsigned dst, unsigned val, int lane)
{
    return ((int)(threadIdx.x & 63) == lane) ? val : dst;
}
__device__ __forceinline__ int clz64_lane(unsigned lo, unsigned hi)  // per-lane clz of (hi:lo), 64 if zero
{
    return hi ? (int)__clz(hi) : (lo ? 32 + (int)__clz(lo) : 64);
}

// Resolve the boundaries of a block of nb rows (lane r holds the ballot mask
// of block row r in (mhi:mlo); `first` = column/offset of lane 0's cell in
// that row).  Fast path: every mask is a contiguous run of lanes 0..last and
// every row moves the boundary by 0 or -1 from the previous one -- the
// structure of Corollary 2.6 / Theorem 4.2 -- so the boundary of row r is the
// run's last cell, found for all rows at once.  Otherwise the previous-cell
// rule is applied row by row (only at rounding-level ties or all-red rows).
// Returns the boundary after the block; lane r of *bq receives row r's.
template <bool TRI_ALLRED>
__device__ __forceinline__ int resolve_block(unsigned mlo, unsigned mhi, int nb, int bc_in, int first,
                                             int first_step, int lo_clamp_lane, int *bq, int tri_i_top)
{
    const int l = threadIdx.x & 63;
    const int fr = first + first_step * l;  // cell of lane 0 in row l
    const int z = clz64_lane(mlo, mhi);
    const int last = fr + 63 - z;           // z = 64 -> fr - 1 (empty)
    const unsigned long long want = (z == 64) ? 0ull : (~0ull >> z);
    const unsigned long long got = ((unsigned long long)mhi << 32) | mlo;
    const int prev = __shfl_up(last, 1, 64);
    const int pv = (l == 0) ? bc_in : prev;
    const bool ok = (l >= nb) || ((got == want) && (last == pv || last == pv - 1) && (last - fr >= lo_clamp_lane));
    if (__ballot(!ok) == 0ull) {
        *bq = last;
        return __builtin_amdgcn_readlane(last, nb - 1);
    }
    // general rule, row by row
    int bc = bc_in;
    int q = 0;
    for (int r = 0; r < nb; ++r) {
        const unsigned long long m = ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)mhi, r) << 32) |
                                     (unsigned)__builtin_amdgcn_readlane((int)mlo, r);
        const int f0 = first + first_step * r;
        if (TRI_ALLRED && bc >= tri_i_top - 2 * r) {  // previous row entirely red (trinomial)
            const int rowlast = tri_i_top - 2 * r - 2 - f0;  // lane of column 2i
            const unsigned long long mm = m & (rowlast >= 63 ? ~0ull : (rowlast < 0 ? 0ull : ((1ull << (rowlast + 1)) - 1ull)));
            bc = mm ? f0 + 63 - (int)__clzll(mm) : f0 - 1;
        } else {
            const int lb = bc - f0;
            if (lb >= 0 && lb < 64) bc -= ((m >> lb) & 1ull) ? 0 : 1;
        }
        q = (l == r) ? bc : q;
    }
    *bq = q;
    return bc;
}

// Binomial: rows i0-1 .. i0-h from row i0, whose red cells are [c0, b]
// (b - c0 + 1 <= BAND); columns >= c0 only.  Writes the red cells of row i0-h
// to dst, the boundary of each row to bnd (may be NULL); returns the last red
// column of row i0-h.  *v0 receives the final value of column c0.
__device__ __forceinline__ ll band_bin(Mp p, ll i0_, ll c0_, ll h_, ll b_, const double *src, double *dst,
                                       ll *bnd, double *v0)
{
    // indices fit in 32 bits (T <= 2^21): scalar 32-bit bookkeeping
    const int i0 = (int)uni(i0_), c0 = (int)uni(c0_), h = (int)uni(h_), b = (int)uni(b_);
    const int l = threadIdx.x & 63;
    const int j = c0 + l;
    const double S = p.S, K = p.K, a = p.a, w0 = p.w0, w1 = p.w1;
    const double u = exp(a);
    double g = (j <= b) ? src[j] : ((j <= i0) ? S * exp((double)(2 * j - i0) * a) - K : 0.0);
    int bc = b;
    for (int k0 = 0; k0 < h; k0 += 64) {
        const int nb = (h - k0) < 64 ? (h - k0) : 64;
        const int itop = i0 - k0;                             // row above the block
        double x = S * exp((double)(2 * j - itop) * a);           // S u^{2j-i}, row itop
        double xn = S * exp((double)(2 * (c0 + BAND) - itop) * a);  // column c0+64
        unsigned mlo = 0, mhi = 0;
#pragma unroll 4
        for (int r = 0; r < nb; ++r) {
            const double gn = dpp_dn1(g, xn - K);  // exercise cell beyond the band
            x *= u;
            xn *= u;
            const double c = fma(w1, gn, w0 * g);
            const double e = x - K;
            g = vmax_f64(c, e);
            // lanes beyond the row's last column (j > i) are outside the tree
            const unsigned long long m = __ballot(c >= e) & row_mask(itop - 1 - r - c0);
            mlo = writelane(mlo, (unsigned)m, r);
            mhi = writelane(mhi, (unsigned)(m >> 32), r);
        }
        int q;
        bc = resolve_block<false>(mlo, mhi, nb, bc, c0, 0, -1, &q, 0);
        if (bnd && l < nb) bnd[itop - 1 - l] = q;
    }
    if (j <= bc) dst[j] = g;
    if (v0 && l == 0) *v0 = g;
    return bc;
}

// Trinomial: as band_bin; row i has columns 0..2i and each cell reads j, j+1,
// j+2.  Below an entirely red row the row shrinks by two cells, and the
// boundary is the row's last red cell.
__device__ __forceinline__ ll band_tri(Mp p, ll i0_, ll c0_, ll h_, ll b_, const double *src, double *dst,
                                       ll *bnd, double *v0)
{
    const int i0 = (int)uni(i0_), c0 = (int)uni(c0_), h = (int)uni(h_), b = (int)uni(b_);
    const int l = threadIdx.x & 63;
    const int j = c0 + l;
    const double S = p.S, K = p.K, a = p.a, w0 = p.w0, w1 = p.w1, w2 = p.w2;
    const double u = exp(a);
    double g = (j <= b) ? src[j] : ((j <= 2 * i0) ? S * exp((double)(j - i0) * a) - K : 0.0);
    int bc = b;
    for (int k0 = 0; k0 < h; k0 += 64) {
        const int nb = (h - k0) < 64 ? (h - k0) : 64;
        const int itop = i0 - k0;
        double x = S * exp((double)(j - itop) * a);           // S u^{j-i}, row itop
        double x1 = S * exp((double)(c0 + BAND - itop) * a);  // column c0+64
        double x2 = x1 * u;                                   // column c0+65
        unsigned mlo = 0, mhi = 0;
#pragma unroll 4
        for (int r = 0; r < nb; ++r) {
            const double g1 = dpp_dn1(g, x1 - K);   // lane 63: column c0+64
            const double g2 = dpp_dn1(g1, x2 - K);  // lane 62: c0+64, lane 63: c0+65
            x *= u;
            x1 *= u;
            x2 *= u;
            const double c = fma(w2, g2, fma(w1, g1, w0 * g));
            const double e = x - K;
            g = vmax_f64(c, e);
            const unsigned long long m = __ballot(c >= e) & row_mask(2 * (itop - 1 - r) - c0);
            mlo = writelane(mlo, (unsigned)m, r);
            mhi = writelane(mhi, (unsigned)(m >> 32), r);
        }
        int q;
        bc = resolve_block<true>(mlo, mhi, nb, bc, c0, 0, -1, &q, 2 * itop);
        if (bnd && l < nb) bnd[itop - 1 - l] = q;
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
// the rightmost cell (the apex when R0 - h = 0).  Here the boundary is the
// last exercise (green) cell; it stays or moves one cell left per step
// (Theorem 4.2).
__device__ __forceinline__ ll band_bsm(Mp p, ll n0_, ll f_, ll h_, ll R0_, const double *src, double *dst,
                                       ll *bnd, double *vr)
{
    // offsets k lie in [-2T-1, T+1]: 32-bit scalar bookkeeping
    const int n0 = (int)uni(n0_), f = (int)uni(f_), h = (int)uni(h_), R0 = (int)uni(R0_);
    const int l = threadIdx.x & 63;
    const int T = (int)p.T;
    const double w0 = p.w0, w1 = p.w1, w2 = p.w2, s0 = p.s0, ds = p.a;
    const double ud = exp(-ds);  // e^{-ds}: one cell to the left
    int base = R0 - 63;
    int k = base + l;
    double v = (k <= f) ? 1.0 - exp(s0 + (double)k * ds) : src[k];
    int fc = f;
    for (int t0 = 0; t0 < h; t0 += 64) {
        const int nb = (h - t0) < 64 ? (h - t0) : 64;
        const int base0 = base;                      // band base before the block
        double x = exp(s0 + (double)(base0 + l) * ds);  // e^{s_k} of the lane's cell before the block
        unsigned mlo = 0, mhi = 0;
#pragma unroll 4
        for (int r = 0; r < nb; ++r) {
            x *= ud;                   // the lane's new cell is one to the left
            const double xm = x * ud;  // e^{s_{k-1}}
            // new cell k needs old cells k-1, k, k+1 = old lanes l-2, l-1, l;
            // lane 0 takes exercise values for the cells left of the band.
            const double vm1 = dpp_up1(v, 1.0 - x);
            const double vm2 = dpp_up1(vm1, 1.0 - xm);
            const double cont = fma(w2, v, fma(w1, vm1, w0 * vm2));
            const double g = 1.0 - x;
            v = vmax_f64(cont, g);
            const unsigned long long m = __ballot(g > cont);
            mlo = writelane(mlo, (unsigned)m, r);
            mhi = writelane(mhi, (unsigned)(m >> 32), r);
        }
        base -= nb;
        int q;
        // row r of the block has lane 0 at cell base0 - 1 - r
        fc = resolve_block<false>(mlo, mhi, nb, fc, base0 - 1, -1, 0, &q, 0);
        if (bnd && l < nb) {
            const int n = n0 + t0 + 1 + l;
            bnd[n] = (q < -(T - n)) ? BSM_NONE : (ll)(q > T - n ? T - n : q);
        }
    }
    k = base + l;
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
    Mp p;
    Stats *st;  // work counters in LDS (updated by lane 0 only)
    double *lo, *hi;  // this option's workspace (doubles) for range checks
    double *arena;
    ll arena_len;
    double2 *scr;
    double2 *lds;
    const double2 *tw;
    const double2 *twl;
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
__device__ __forceinline__ ll solve_trapezoid(const Ctx &cx, Frame root, Frame *stk, int *sp_sh, ll *ret_sh,
                              int *err_sh, ll *leaf_sh)
{
    const Mp d = cx.p;
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
        fr.r0 = uni(fr.r0);
        fr.c0 = uni(fr.c0);
        fr.h = uni(fr.h);
        fr.b = uni(fr.b);
        fr.aoff = uni(fr.aoff);
        const ll rv = uni(*ret_sh);
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
                        const ll tb = clk();
                        if (tid < 64) {
                            const ll r = (d.model == BINOMIAL)
                                             ? band_bin(d, i0, c0, h, b, fr.src, fr.dst, cx.bnd, nullptr)
                                             : band_tri(d, i0, c0, h, b, fr.src, fr.dst, cx.bnd, nullptr);
                            if (tid == 0) {
                                *leaf_sh = r;
                                cx.st->band_rows += h;
                                cx.st->cyc_band += clk() - tb;
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
                        correlate(cx.st, d, fr.src + c0, nred, h1, (span == 1) ? 0 : h1, nred - span * h1,
                                      mid + c0, cx.scr, cx.lds, cx.tw, cx.twl);
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
                        correlate(cx.st, d, fr.mid + c0, n2, h2, (span == 1) ? 0 : h2, n2 - span * h2,
                                      fr.dst + c0, cx.scr, cx.lds, cx.tw, cx.twl);
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
                        const ll tb = clk();
                        if (tid < 64) {
                            const ll r = band_bsm(d, n, f, h, f + 2 * h, fr.src, fr.dst, cx.bnd, nullptr);
                            if (tid == 0) {
                                *leaf_sh = r;
                                cx.st->band_rows += h;
                                cx.st->cyc_band += clk() - tb;
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
                        correlate(cx.st, d, fr.src + f + 1, 2 * h, h1, h1, 2 * h - 2 * h1, mid + f + 1 + h1,
                                      cx.scr, cx.lds, cx.tw, cx.twl);
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
                    correlate(cx.st, d, fr.mid + fp + 1, nin, h2, h2, nin - 2 * h2, fr.dst + fp + 1 + h2,
                                  cx.scr, cx.lds, cx.tw, cx.twl);
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
__device__ __forceinline__ double drive_lattice(const Ctx &cx, double *rowA, double *rowB, Frame *stk, int *sp_sh,
                                ll *ret_sh, int *err_sh, ll *leaf_sh, ll *red_sh, double *val_sh)
{
    const Mp d = cx.p;
    const ll T = d.T;
    const int tid = threadIdx.x;
    const bool bin = d.model == BINOMIAL;
    const ll wT = bin ? T : 2 * T;  // last column of row T
    // Expiry row T (red = out of the money: G^red = 0 >= G^green) and row T-1.
    const ll tr0 = clk();
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
    if (tid == 0) cx.st->cyc_rows += clk() - tr0;
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
        correlate(cx.st, d, src, b + 1, hh, bin ? 0 : hh, 1, val_sh, cx.scr, cx.lds, cx.tw, cx.twl, beta, tc);
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
            const ll tb = clk();
            if (tid < 64) {
                if (bin) band_bin(d, i0, 0, i0, b, src, dst, cx.bnd, val_sh);
                else band_tri(d, i0, 0, i0, b, src, dst, cx.bnd, val_sh);
            }
            __syncthreads();
            if (tid == 0) {
                cx.st->band_rows += i0;
                cx.st->cyc_band += clk() - tb;
            }
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

__device__ __forceinline__ double drive_bsm(const Ctx &cx, double *rowA, double *rowB, Frame *stk, int *sp_sh,
                            ll *ret_sh, int *err_sh, ll *leaf_sh, ll *red_sh, double *val_sh)
{
    const Mp d = cx.p;
    const ll T = d.T;
    const int tid = threadIdx.x;
    const ll NONE = LLONG_MIN;
    const ll tr0 = clk();
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
    if (tid == 0) cx.st->cyc_rows += clk() - tr0;
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
            correlate(cx.st, d, src + L, R - L + 1, hh, hh, 1, val_sh, cx.scr, cx.lds, cx.tw, cx.twl);
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
            const ll tb = clk();
            if (tid < 64) band_bsm(d, n, f, T - n, R, src, dst, cx.bnd, val_sh);
            __syncthreads();
            if (tid == 0) {
                cx.st->band_rows += T - n;
                cx.st->cyc_band += clk() - tb;
            }
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
        correlate(cx.st, d, src + f + 1, w, h, h, w - 2 * h, dst + f + 1 + h, cx.scr, cx.lds, cx.tw, cx.twl);
        n += h;
        R -= h;
        L += h;
        f = fn;
        double *t = src;
        src = dst;
        dst = t;
    }
}

__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(1, 1))) solve_kernel(const Desc *__restrict__ descs, char *ws,
                                                   const double2 *__restrict__ tw, double *price,
                                                   ll *bnd, ll bnd_stride, int32_t *err, Stats *stats)
{
    __shared__ double2 lds[NLDS];
    __shared__ double2 twl[NLDS / 2];
    __shared__ Frame stk[MAXD];
    __shared__ int sp_sh, err_sh;
    __shared__ ll ret_sh, leaf_sh, red_sh[WG / 64];
    __shared__ double val_sh;
    __shared__ Stats st_sh;

    const Desc d = descs[blockIdx.x];
    if (d.model < 0) {  // rejected on the host: no work, price NaN
        if (threadIdx.x == 0) {
            price[d.out_index] = NAN;
            stats[d.out_index] = Stats{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        }
        return;
    }
    char *base = ws + d.ws_off;
    double *rowA = (double *)base;
    double *rowB = rowA + d.row_len;
    double *arena = rowB + d.row_len;
    double2 *scr = (double2 *)(arena + d.arena_len);
    Ctx cx;
    cx.p = make_mp(d);
    cx.lo = rowA;
    cx.hi = (double *)(scr + d.nfft);
    cx.arena = arena;
    cx.arena_len = d.arena_len;
    cx.scr = scr;
    cx.lds = lds;
    cx.tw = tw;
    cx.twl = twl;
    for (int t = threadIdx.x; t < NLDS / 2; t += WG) twl[t] = tw[(ll)t << (LG_TW - LG_NLDS)];
    cx.bnd = bnd ? bnd + d.out_index * bnd_stride : nullptr;
    cx.st = &st_sh;
    if (threadIdx.x == 0) {
        err_sh = 0;
        ret_sh = 0;
        st_sh = Stats{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    }
    __syncthreads();
    const ll ttot = clk();
    double p;
    if (d.model == BSM)
        p = drive_bsm(cx, rowA, rowB, stk, &sp_sh, &ret_sh, &err_sh, &leaf_sh, red_sh, &val_sh);
    else
        p = drive_lattice(cx, rowA, rowB, stk, &sp_sh, &ret_sh, &err_sh, &leaf_sh, red_sh, &val_sh);
    __syncthreads();
    if (threadIdx.x == 0) {
        price[d.out_index] = err_sh ? NAN : p;
        if (err) err[d.out_index] = err_sh;
        st_sh.cyc_total = clk() - ttot;
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
