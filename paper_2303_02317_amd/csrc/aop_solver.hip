// aop_solver.hip -- gfx950 kernels of the FFT nonlinear-stencil pricer.
//
// One persistent launch prices a batch of options.  Each workgroup (256
// lanes, 4 wave64) claims an option and drives it:
//   1. computes the expiry row and the first backward row directly (the
//      corollary relating consecutive boundaries only holds below the top row),
//   2. runs the trapezoid decomposition (Sec. 2.3 "Partitioning the triangle",
//      Sec. 3 / appendix A.3, Sec. 4.3): each trapezoid is solved recursively
//      ("Solving a trapezoid"); guaranteed-continuation (red) segments are
//      advanced h rows at once by a correlation with the h-step stencil kernel,
//      by FFT with the kernel's spectrum evaluated per bin in closed form (FP64)
//      or, for short kernels, by direct stepping of the linear stencil,
//   3. solves the base cases with a one-wave band walker that applies the
//      max(continuation, exercise) stencil directly, one lane per cell, and
//      finds each row's boundary with a wave ballot.
// Correlations are published as tiled jobs in a work pool that every
// workgroup without an option of its own (and each driver, for its own jobs)
// takes tiles from, so that one option's transforms spread over the chip
// while its driver walks the band.  The recursion runs on an explicit stack in
// LDS; control flow is uniform across a workgroup.  Every range a step touches
// is checked against the option's workspace first; a failed check records an
// error and prices NaN.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <math.h>
#include <stdint.h>

#include "aop_internal.h"

namespace aop {

#define WG 256
#define NLDS 2048  // complex doubles staged in LDS per FFT tile (32 KB)
#define LG_NLDS 11
#define NLDS64 4096  // FP64 transforms of up to this many points run whole in LDS (64 KB)
#define LG_NLDS64 12
#define MAXD 48    // recursion depth bound (log2 of 2^22 plus slack)
#define BAND 64    // cells held by the Bermudan band walker (one per lane)
#define BAND2 128  // cells held by the lattice and BSM band walkers (two per lane)

typedef long long ll;

// Model parameters, passed by value so that they live in registers.
struct Mp {
    int model, no_green, ex_every;  // ex_every: 1 American, 0 European, d >= 2 Bermudan (rows (T - i) % d == 0)
    ll T;
    double S, K, a, s0, w0, w1, w2;
};
__device__ __forceinline__ Mp make_mp(const Desc &d)
{
    Mp p;
    p.model = d.model;
    p.T = d.T;
    p.no_green = d.no_green;
    p.ex_every = d.ex_every;
    p.S = d.S;
    p.K = d.K;
    p.a = d.a;
    p.s0 = d.s0;
    p.w0 = d.w0;
    p.w1 = d.w1;
    p.w2 = d.w2;
    return p;
}

// Cells of a band leaf: the lattice and BSM walkers hold two per lane, the
// Bermudan walker one.
__device__ __forceinline__ ll band_width(const Mp &p)
{
    return (p.model == BSM || p.ex_every <= 1) ? BAND2 : BAND;
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
// round trips.  twl holds e^{-2 pi i t / 4096}, t <= 2048 (LDS); both are
// addressed through px().
// w * e^{-2 pi i p / 2^(t+1)}, p < 2^t <= 4: one of the 8th roots of unity
// (t and p are constants after unrolling, so this folds to a few operations).
// Index into the LDS transform buffer and trig table: one padding element
// after every 8 complex values, so that the strided passes of a transform
// (stride 8 .. 64 elements at the last stages) fall on different banks.
__device__ __forceinline__ int px(int i) { return i + (i >> 3); }

__device__ __forceinline__ double2 rot_root(double2 w, int t, int p)
{
    if (p == 0) return w;
    if (t == 1 || p == 2) return make_double2(w.y, -w.x);  // times -i
    const double c = 0.70710678118654752440;            // sqrt(1/2)
    const double P = c * (w.x + w.y), M = c * (w.y - w.x);
    return p == 1 ? make_double2(P, M) : make_double2(M, -P);  // times e^{-i pi/4}, e^{-3 i pi/4}
}

// The twiddle of stage s = s_lo + t for the element at q 2^s_lo + j of its
// half-block is e^{-2 pi i j / 2^(s+1)} -- one table value per stage and
// thread -- times a root of unity fixed by q (rot_root).
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
        double2 v[G], om[K];
#pragma unroll
        for (int q = 0; q < G; ++q) v[q] = x[px(base + (q << s_lo))];
#pragma unroll
        for (int t = 0; t < K; ++t) om[t] = twl[px(j << (11 - s_lo - t))];
        if (!INV) {
#pragma unroll
            for (int t = K - 1; t >= 0; --t) {
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    if (q & (1 << t)) continue;
                    const double2 w = rot_root(om[t], t, q & ((1 << t) - 1));
                    const double2 u = v[q], z = v[q + (1 << t)];
                    v[q] = make_double2(u.x + z.x, u.y + z.y);
                    v[q + (1 << t)] = cmul(make_double2(u.x - z.x, u.y - z.y), w);
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < K; ++t) {
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    if (q & (1 << t)) continue;
                    const double2 w = rot_root(om[t], t, q & ((1 << t) - 1));
                    const double2 u = v[q], z = cmulc(v[q + (1 << t)], w);
                    v[q] = make_double2(u.x + z.x, u.y + z.y);
                    v[q + (1 << t)] = make_double2(u.x - z.x, u.y - z.y);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < G; ++q) x[px(base + (q << s_lo))] = v[q];
    }
    __syncthreads();
}

__device__ void lds_dif(double2 *x, int lg, int nb, const double2 *twl, int rk)
{
    int s_hi = lg - 1;
    while (s_hi >= 0) {
        const int k = s_hi + 1 >= rk ? rk : s_hi + 1;
        const int s_lo = s_hi - k + 1;
        if (k == 3) lds_pass<3, false>(x, lg, nb, s_lo, twl);
        else if (k == 2) lds_pass<2, false>(x, lg, nb, s_lo, twl);
        else lds_pass<1, false>(x, lg, nb, s_lo, twl);
        s_hi = s_lo - 1;
    }
}

__device__ void lds_dit_inv(double2 *x, int lg, int nb, const double2 *twl, int rk)
{
    int s_lo = 0;
    while (s_lo < lg) {
        const int k = lg - s_lo >= rk ? rk : lg - s_lo;
        if (k == 3) lds_pass<3, true>(x, lg, nb, s_lo, twl);
        else if (k == 2) lds_pass<2, true>(x, lg, nb, s_lo, twl);
        else lds_pass<1, true>(x, lg, nb, s_lo, twl);
        s_lo += k;
    }
}

// ------------------------------------------- split-precision (FP32 hi/lo)
// The mixed-precision transforms hold every value as an unevaluated sum of
// two FP32 numbers, hi + lo with |lo| <= ulp(hi)/2, and use error-free
// transformations: two-sum for additions and the FMA-exact product for
// multiplications, so each operation is exact up to a rounding of order
// 2^-48 relative; all arithmetic is FP32.  Twiddles come split the same way.
// Contraction is disabled inside these helpers: the two-sum identities need
// every intermediate rounded exactly as written.
struct CF {
    float rh, rl, ih, il;  // real hi/lo, imaginary hi/lo
};

__device__ __forceinline__ void ff_two_sum(float a, float b, float &s, float &e)
{
#pragma clang fp contract(off)
    s = a + b;
    const float v = s - a;
    e = (a - (s - v)) + (b - v);
}
__device__ __forceinline__ void ff_norm(float s, float e, float &h, float &l)
{
#pragma clang fp contract(off)
    h = s + e;
    l = e - (h - s);
}
__device__ __forceinline__ void ff_add(float ah, float al, float bh, float bl, float &h, float &l)
{
#pragma clang fp contract(off)
    float s, e;
    ff_two_sum(ah, bh, s, e);
    e += al + bl;
    ff_norm(s, e, h, l);
}
__device__ __forceinline__ CF cf_add(const CF &a, const CF &b)
{
    CF r;
    ff_add(a.rh, a.rl, b.rh, b.rl, r.rh, r.rl);
    ff_add(a.ih, a.il, b.ih, b.il, r.ih, r.il);
    return r;
}
__device__ __forceinline__ CF cf_sub(const CF &a, const CF &b)
{
    CF r;
    ff_add(a.rh, a.rl, -b.rh, -b.rl, r.rh, r.rl);
    ff_add(a.ih, a.il, -b.ih, -b.il, r.ih, r.il);
    return r;
}
// x*y + u*v for split operands, with sy = +1 or -1 on the second product.
__device__ __forceinline__ void ff_dot2(float xh, float xl, float yh, float yl, float uh, float ul, float vh,
                                        float vl, float sg, float &h, float &l)
{
#pragma clang fp contract(off)
    const float p1 = xh * yh;
    const float e1 = fmaf(xh, yh, -p1);
    const float p2 = sg * (uh * vh);
    const float e2 = sg * fmaf(uh, vh, -(uh * vh));
    float s, e;
    ff_two_sum(p1, p2, s, e);
    e += (e1 + e2) + (fmaf(xh, yl, xl * yh) + sg * fmaf(uh, vl, ul * vh));
    ff_norm(s, e, h, l);
}
__device__ __forceinline__ CF cf_mul(const CF &a, const CF &w)  // a * w
{
    CF r;
    ff_dot2(a.rh, a.rl, w.rh, w.rl, a.ih, a.il, w.ih, w.il, -1.0f, r.rh, r.rl);
    ff_dot2(a.rh, a.rl, w.ih, w.il, a.ih, a.il, w.rh, w.rl, 1.0f, r.ih, r.il);
    return r;
}
__device__ __forceinline__ CF cf_mulc(const CF &a, const CF &w)  // a * conj(w)
{
    CF r;
    ff_dot2(a.rh, a.rl, w.rh, w.rl, a.ih, a.il, w.ih, w.il, 1.0f, r.rh, r.rl);
    ff_dot2(a.ih, a.il, w.rh, w.rl, a.rh, a.rl, w.ih, w.il, -1.0f, r.ih, r.il);
    return r;
}
__device__ __forceinline__ CF cf_from(double re, double im)
{
    CF r;
    r.rh = (float)re;
    r.rl = (float)(re - (double)r.rh);
    r.ih = (float)im;
    r.il = (float)(im - (double)r.ih);
    return r;
}
__device__ __forceinline__ double2 cf_to(const CF &a)
{
    return make_double2((double)a.rh + (double)a.rl, (double)a.ih + (double)a.il);
}
__device__ __forceinline__ CF ld_cf(const float4 *p)
{
    const float4 v = *p;
    return CF{v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ void st_cf(float4 *p, const CF &a) { *p = make_float4(a.rh, a.rl, a.ih, a.il); }

// The LDS passes of lds_pass in split precision (twf: split twiddles).
template <int K, bool INV>
__device__ __forceinline__ void lds_pass_ff(float4 *x, int lg, int nb, int s_lo, const float4 *twf)
{
    constexpr int G = 1 << K;
    const int n = 1 << lg;
    const int s_hi = s_lo + K - 1;
    const int per = n >> K;
    const int groups = nb * per;
    const int jmask = (1 << s_lo) - 1;
    for (int gi = threadIdx.x; gi < groups; gi += WG) {
        const int b = gi / per;
        const int r = gi - b * per;
        const int j = r & jmask;
        const int blk = r >> s_lo;
        const int base = b * n + (blk << (s_hi + 1)) + j;
        CF v[G];
#pragma unroll
        for (int q = 0; q < G; ++q) v[q] = ld_cf(x + base + (q << s_lo));
        if (!INV) {
#pragma unroll
            for (int t = K - 1; t >= 0; --t) {
                const int s = s_lo + t;
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    if (q & (1 << t)) continue;
                    const int jj = ((q & ((1 << t) - 1)) << s_lo) + j;
                    const CF w = ld_cf(twf + (jj << (10 - s)));
                    const CF u = v[q], z = v[q + (1 << t)];
                    v[q] = cf_add(u, z);
                    v[q + (1 << t)] = cf_mul(cf_sub(u, z), w);
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
                    const CF w = ld_cf(twf + (jj << (10 - s)));
                    const CF u = v[q], z = cf_mulc(v[q + (1 << t)], w);
                    v[q] = cf_add(u, z);
                    v[q + (1 << t)] = cf_sub(u, z);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < G; ++q) st_cf(x + base + (q << s_lo), v[q]);
    }
    __syncthreads();
}

__device__ void lds_dif_ff(float4 *x, int lg, int nb, const float4 *twf)
{
    int s_hi = lg - 1;
    while (s_hi >= 0) {
        const int k = s_hi + 1 >= 3 ? 3 : s_hi + 1;
        const int s_lo = s_hi - k + 1;
        if (k == 3) lds_pass_ff<3, false>(x, lg, nb, s_lo, twf);
        else if (k == 2) lds_pass_ff<2, false>(x, lg, nb, s_lo, twf);
        else lds_pass_ff<1, false>(x, lg, nb, s_lo, twf);
        s_hi = s_lo - 1;
    }
}

__device__ void lds_dit_inv_ff(float4 *x, int lg, int nb, const float4 *twf)
{
    int s_lo = 0;
    while (s_lo < lg) {
        const int k = lg - s_lo >= 3 ? 3 : lg - s_lo;
        if (k == 3) lds_pass_ff<3, true>(x, lg, nb, s_lo, twf);
        else if (k == 2) lds_pass_ff<2, true>(x, lg, nb, s_lo, twf);
        else lds_pass_ff<1, true>(x, lg, nb, s_lo, twf);
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

// Trig values of a bin from the LDS table (e^{-2 pi i t / 4096}, t <= 2048).
__device__ __forceinline__ double2 twl_at(const double2 *twl, int t)  // any t in [0, 4096)
{
    if (t <= 2048) return twl[px(t)];
    const double2 w = twl[px(t - 2048)];  // e^{-i pi} e^{-2 pi i (t - 2048) / 4096}
    return make_double2(-w.x, -w.y);
}
// Largest transform (log2 of its points) that runs whole in LDS.
__device__ __forceinline__ int lds_lg(int prec) { return prec ? LG_NLDS : LG_NLDS64; }

// Bin f of a transform of 2^lgN <= 4096 points: theta = 2 pi f / N, f <= N / 2.
__device__ __forceinline__ void bin_trig_lds(const double2 *twl, const double2 *__restrict__ tw, ll f, int lgN,
                                             double &cs, double &sn, double &sh)
{
    const double2 e = twl[px((int)(f << (12 - lgN)))];
    cs = e.x;
    sn = -e.y;
    if (lgN <= LG_NLDS) sh = twl[px((int)(f << (11 - lgN)))].y;
    else sh = tw[f << (LG_TW - lgN - 1)].y;  // 4096 points: theta / 2 from the 2^22 table
}
// The same for transforms of up to 2048 points (the LDS table alone).
__device__ __forceinline__ void bin_trig_lds11(const double2 *twl, ll f, int lgN, double &cs, double &sn, double &sh)
{
    const double2 e = twl[px((int)(f << (12 - lgN)))];
    cs = e.x;
    sn = -e.y;
    sh = twl[px((int)(f << (11 - lgN)))].y;
}
// Bin k1 + N1 k2 of a four-step transform (N = N1 * 2048): r1 = e^{-2 pi i k1/N}
// and r2 = e^{-i pi k1/N} are the tile's row factors, the rest comes from LDS.
__device__ __forceinline__ void bin_trig_rows(const double2 *twl, double2 r1, double2 r2, int k2, double &cs,
                                              double &sn, double &sh)
{
    const double2 a = twl_at(twl, 2 * k2);
    const double2 e = cmul(r1, a);
    cs = e.x;
    sn = -e.y;
    sh = cmul(r2, twl[px(k2)]).y;
}
// e^{-2 pi i m / N}, m < N (four-step column twiddles), by sincospi in FP64.
__device__ __forceinline__ double2 twiddle_n(ll m, int lgN)
{
    double sv, cv;
    sincospi((double)(2 * m) / (double)(ll(1) << lgN), &sv, &cv);
    return make_double2(cv, -sv);
}
// Four-step column twiddles from tables: for N = 4096 * 2^s, m = m_hi 2^s +
// m_lo gives e^{-2 pi i m_hi / 4096} (the LDS trig table) times
// e^{-2 pi i m_lo / N}, m_lo < 2^s, from the tile's small table twx (copied
// from the 2^22-point global table into LDS above the tile's values).
#define TWX_OFF 2560
// Staging area of a private whole-LDS correlation's input (up to 2048
// doubles), above the small twiddle table: see conv_submit.
#define STG_OFF 3584
static_assert(STG_OFF >= TWX_OFF + (1 << (LG_TW - LG_NLDS - 1)) && STG_OFF + NLDS / 2 <= NLDS64 + NLDS64 / 8,
              "the staging area lies above the column tiles' table, inside the FP64 LDS buffer");
static_assert(TWX_OFF >= NLDS + NLDS / 8 && TWX_OFF + (1 << (LG_TW - LG_NLDS - 1)) <= NLDS64 + NLDS64 / 8,
              "the small twiddle table lies above a column tile's padded values, inside the FP64 LDS buffer");
__device__ __forceinline__ void fill_twx(double2 *twx, int lgN, const double2 *__restrict__ tw)
{
    const int s = lgN - (LG_NLDS + 1);
    for (int r = threadIdx.x; r < (1 << s); r += WG) twx[r] = tw[(ll)r << (LG_TW - lgN)];
}
__device__ __forceinline__ double2 twiddle_col(ll m, int lgN, const double2 *twl, const double2 *twx)
{
    const int s = lgN - (LG_NLDS + 1);
    const double2 hi = twl_at(twl, (int)(m >> s));
    return s == 0 ? hi : cmul(hi, twx[m & ((ll(1) << s) - 1)]);
}

// cs, sn: cos and sin of theta; sh: +-sin(theta/2) (only its square is used).
__device__ __forceinline__ double2 kernel_power(const Spec &q, double cs, double sn, double sh)
{
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
// A row value that overflowed FP64 (the top of a lattice row when V sqrt(E T)
// exceeds ~709) lies so far above the strike that the risk-neutral weight of
// reaching it is below e^{-T/4}; without exercise (Y = 0 or a European option)
// nothing stops the plain induction from carrying the infinity to the root, so
// such a value is left out of the correlation (its product with its weight is
// far below the rounding of the result).
__device__ __forceinline__ double tilt_in(double x, double beta, ll t, double tc)
{
    if (!(x < INFINITY)) return 0.0;
    return (beta == 0.0 || x == 0.0) ? x : x * exp(-beta * ((double)t - tc));
}
// The untilting factor e^{beta (m - tc)} is applied in one piece: split into
// e^{beta m} and e^{-beta tc} each part can overflow once beta tc > 709 (a
// lattice row of T ~ 2^20 cells with V sqrt(E T) above ~700).
__device__ __forceinline__ double tilt_out(double y, double beta, ll m, double tc)
{
    return beta == 0.0 ? y : y * exp(beta * ((double)m - tc));
}

// A correlation job computes dst[t] = (x (*) W^(h))[out_off + t], t < n_out,
// where x = src[0..n_in) zero-padded to N = 2^lgN and (*) is the circular
// correlation with the h-step stencil kernel; for out_off + n_out <= n_in -
// span the window never wraps, so the result is the linear one.  Kinds:
//   K_DIRECT  h applications of the one-step linear stencil in one wave;
//   K_LDS     one transform in LDS (N <= 2048);
//   K_4STEP   N = N1 x 2048 through the global scratch `scr` (N complex), in
//             three phases of N1 tiles each:
//     phase 0, tile t: length-N1 column transforms of columns [tC, tC + C)
//                      (C = 2048 / N1) of the N1 x 2048 row-major view, times
//                      w_N^{n2 k1}; rows are left in bit-reversed k1 order;
//     phase 1, tile t: row t: forward length-2048 transform, product with the
//                      kernel power at frequency k1 + N1 k2, inverse;
//     phase 2, tile t: conjugate twiddle, inverse column transforms, output.
// Tiles of one phase are independent; a phase starts once the previous one
// has completed.  With beta != 0 the input is tilted, x~_t = x_t e^{-beta (t -
// tc)}, the kernel spectrum is tilted to match and the output untilted, y_m =
// y~_m e^{beta (m - tc)}, so that a segment growing like e^{beta t} is
// transformed at uniform relative precision.
enum { K_DIRECT = 0, K_LDS = 1, K_4STEP = 2 };

struct JobArgs {
    const double *src;
    double *dst;
    double2 *scr;
    ll n_in, h, out_off, n_out;
    double beta, tc;
    int desc, lgN, kind, ntile, nph, prec;  // prec: 0 FP64, 1 split FP32
    int radix;                               // FP64 LDS passes of radix 2^radix (2 or 3)
    int cached;                              // K_LDS: 1 if scr holds the job's kernel spectrum (bins 0 .. N/2)
};
static_assert(sizeof(JobArgs) == 104, "job arguments are 104 bytes");

__device__ __forceinline__ JobArgs uni_args(JobArgs a)
{
    JobArgs u = a;
    u.n_in = uni(a.n_in);
    u.h = uni(a.h);
    u.out_off = uni(a.out_off);
    u.n_out = uni(a.n_out);
    u.desc = __builtin_amdgcn_readfirstlane(a.desc);
    u.lgN = __builtin_amdgcn_readfirstlane(a.lgN);
    u.kind = __builtin_amdgcn_readfirstlane(a.kind);
    u.ntile = __builtin_amdgcn_readfirstlane(a.ntile);
    u.nph = __builtin_amdgcn_readfirstlane(a.nph);
    u.prec = __builtin_amdgcn_readfirstlane(a.prec);
    u.radix = __builtin_amdgcn_readfirstlane(a.radix);
    u.cached = __builtin_amdgcn_readfirstlane(a.cached);
    return u;
}

// One whole transform in LDS (FP64, N <= 4096).
__device__ __forceinline__ void tile_lds(const Mp &p, const JobArgs &j, double2 *lds, const double2 *__restrict__ tw,
                                         const double2 *twl, const double2 *spec = nullptr)
{
    const int lgN = j.lgN;
    const ll N = ll(1) << lgN;
    const double invN = 1.0 / (double)N;
    const Spec q = make_spec(p, j.h, j.beta, 0.0);
    const int tid = threadIdx.x;
    // unrolled so that several global loads are in flight at once
    if (j.cached & 2) {
        // the input pairs were loaded into the staging area when the job was
        // submitted (direct global-to-LDS loads): wait for them, then spread
        const double *stg = (const double *)(lds + STG_OFF);
        const ll staged = j.n_in & ~ll(1);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        for (int t = tid; t < N; t += WG)
            lds[px(t)] = make_double2(t < staged ? stg[t] : (t < j.n_in ? j.src[t] : 0.0), 0.0);
    } else if (j.beta == 0.0) {
#pragma unroll 4
        for (int t = tid; t < N; t += WG) lds[px(t)] = make_double2(t < j.n_in ? j.src[t] : 0.0, 0.0);
    } else {
        for (int t = tid; t < N; t += WG)
            lds[px(t)] = make_double2(t < j.n_in ? tilt_in(j.src[t], j.beta, t, j.tc) : 0.0, 0.0);
    }
    __syncthreads();
    lds_dif(lds, lgN, 1, twl, j.radix);
    // P(-theta) = conj(P(theta)): evaluate f <= N/2 and apply to both mirrors.
    if (spec) {
#pragma unroll 4
        for (int f = tid; f <= N / 2; f += WG) {
            const double2 m = spec[f];
            const unsigned t1 = bitrev((unsigned)f, lgN), t2 = bitrev((unsigned)((N - f) & (N - 1)), lgN);
            lds[px(t1)] = cmul(lds[px(t1)], m);
            if (t2 != t1) lds[px(t2)] = cmulc(lds[px(t2)], m);
        }
    } else {
        for (int f = tid; f <= N / 2; f += WG) {
            double cs, sn, sh;
            bin_trig_lds(twl, tw, f, lgN, cs, sn, sh);
            const double2 m = kernel_power(q, cs, sn, sh);
            const unsigned t1 = bitrev((unsigned)f, lgN), t2 = bitrev((unsigned)((N - f) & (N - 1)), lgN);
            lds[px(t1)] = cmul(lds[px(t1)], m);
            if (t2 != t1) lds[px(t2)] = cmulc(lds[px(t2)], m);
        }
    }
    __syncthreads();
    lds_dit_inv(lds, lgN, 1, twl, j.radix);
    for (ll t = tid; t < j.n_out; t += WG)
        j.dst[t] = tilt_out(lds[px((int)(j.out_off + t))].x * invN, j.beta, j.out_off + t, j.tc);
    __syncthreads();
}

__device__ __forceinline__ void tile_col_fwd(const JobArgs &j, int tile, double2 *lds, const double2 *__restrict__ tw,
                                             const double2 *twl)
{
    const int lgN = j.lgN, lg2 = LG_NLDS, lg1 = lgN - lg2;
    const ll N = ll(1) << lgN, N2 = ll(1) << lg2;
    const int N1 = 1 << lg1, lgC = lg2 - lg1, C = 1 << lgC;
    const ll n20 = (ll)tile * C;
    const int tid = threadIdx.x;
    // unrolled so that several global loads are in flight at once
#pragma unroll 4
    for (int t = tid; t < NLDS; t += WG) {
        const int c = t & (C - 1), n1 = t >> lgC;
        const ll idx = (ll)n1 * N2 + n20 + c;
        lds[px(c * N1 + n1)] = make_double2(idx < j.n_in ? j.src[idx] : 0.0, 0.0);
    }
    if (j.beta != 0.0)  // the same elements, in the same threads: no barrier needed in between
        for (int t = tid; t < NLDS; t += WG) {
            const int c = t & (C - 1), n1 = t >> lgC;
            lds[px(c * N1 + n1)].x = tilt_in(lds[px(c * N1 + n1)].x, j.beta, (ll)n1 * N2 + n20 + c, j.tc);
        }
    double2 *twx = lds + TWX_OFF;
    fill_twx(twx, lgN, tw);
    __syncthreads();
    lds_dif(lds, lg1, C, twl, j.radix);
    for (int t = tid; t < NLDS; t += WG) {
        const int c = t & (C - 1), p1 = t >> lgC;
        const ll k1 = bitrev(p1, lg1), n2 = n20 + c;
        const double2 w = twiddle_col((n2 * k1) & (N - 1), lgN, twl, twx);
        j.scr[(ll)p1 * N2 + n2] = cmul(lds[px(c * N1 + p1)], w);
    }
    __syncthreads();
}

__device__ __forceinline__ void tile_rows(const Mp &p, const JobArgs &j, int tile, double2 *lds,
                                          const double2 *__restrict__ tw, const double2 *twl,
                                          const double2 *spec = nullptr)
{
    const int lgN = j.lgN, lg2 = LG_NLDS, lg1 = lgN - lg2;
    const ll N2 = ll(1) << lg2;
    const Spec q = make_spec(p, j.h, j.beta, 0.0);
    const int tid = threadIdx.x;
    const int p1 = tile;
    const ll k1 = bitrev(p1, lg1);
    double2 *row = j.scr + (ll)p1 * N2;
#pragma unroll 4
    for (int t = tid; t < N2; t += WG) lds[px(t)] = row[t];
    __syncthreads();
    lds_dif(lds, lg2, 1, twl, j.radix);
    if (spec) {
        // bin f = k1 + N1 k2; above N/2 the mirror's conjugate
        const ll N = ll(1) << lgN;
#pragma unroll 4
        for (int k2 = tid; k2 < N2; k2 += WG) {
            const int t = (int)bitrev(k2, lg2);
            const ll f = k1 + ((ll)k2 << lg1);
            const double2 e = spec[f <= N / 2 ? f : N - f];
            lds[px(t)] = cmul(lds[px(t)], f <= N / 2 ? e : make_double2(e.x, -e.y));
        }
    } else {
        double sr, cr;
        sincospi((double)(2 * k1) / (double)(ll(1) << lgN), &sr, &cr);
        const double2 r1 = make_double2(cr, -sr);
        sincospi((double)k1 / (double)(ll(1) << lgN), &sr, &cr);
        const double2 r2 = make_double2(cr, -sr);
        // bins in natural order, so that the lanes of a wave hold neighbouring
        // frequencies: the significant bins (|P|^h above e^-60, a narrow band
        // around theta = 0 for long kernels) then fall in a few waves, and the
        // others skip the transcendental part together
        for (int k2 = tid; k2 < N2; k2 += WG) {
            const int t = (int)bitrev(k2, lg2);
            double cs, sn, sh;
            bin_trig_rows(twl, r1, r2, k2, cs, sn, sh);
            lds[px(t)] = cmul(lds[px(t)], kernel_power(q, cs, sn, sh));
        }
    }
    __syncthreads();
    lds_dit_inv(lds, lg2, 1, twl, j.radix);
    for (int t = tid; t < N2; t += WG) row[t] = lds[px(t)];
    __syncthreads();
}

__device__ __forceinline__ void tile_col_inv(const JobArgs &j, int tile, double2 *lds, const double2 *__restrict__ tw,
                                             const double2 *twl)
{
    const int lgN = j.lgN, lg2 = LG_NLDS, lg1 = lgN - lg2;
    const ll N = ll(1) << lgN, N2 = ll(1) << lg2;
    const int N1 = 1 << lg1, lgC = lg2 - lg1, C = 1 << lgC;
    const double invN = 1.0 / (double)N;
    const ll n20 = (ll)tile * C;
    const int tid = threadIdx.x;
    // loads first (unrolled: several in flight), then the twiddles in place
#pragma unroll 4
    for (int t = tid; t < NLDS; t += WG) {
        const int c = t & (C - 1), p1 = t >> lgC;
        lds[px(c * N1 + p1)] = j.scr[(ll)p1 * N2 + n20 + c];
    }
    double2 *twx = lds + TWX_OFF;
    fill_twx(twx, lgN, tw);
    __syncthreads();
    for (int t = tid; t < NLDS; t += WG) {  // the same elements, in the same threads
        const int c = t & (C - 1), p1 = t >> lgC;
        const ll k1 = bitrev(p1, lg1), n2 = n20 + c;
        const double2 w = twiddle_col((n2 * k1) & (N - 1), lgN, twl, twx);
        lds[px(c * N1 + p1)] = cmulc(lds[px(c * N1 + p1)], w);
    }
    __syncthreads();
    lds_dit_inv(lds, lg1, C, twl, j.radix);
    for (int t = tid; t < NLDS; t += WG) {
        const int c = t & (C - 1), n1 = t >> lgC;
        const ll idx = (ll)n1 * N2 + n20 + c;
        if (idx >= j.out_off && idx < j.out_off + j.n_out)
            j.dst[idx - j.out_off] = tilt_out(lds[px(c * N1 + n1)].x * invN, j.beta, idx, j.tc);
    }
    __syncthreads();
}

// The same tiles in split precision (JobArgs::prec == 1): rows enter as FP64,
// are split to hi/lo FP32 and transformed with the split arithmetic above;
// the kernel power (FP64) and the four-step twiddles (from the FP64 table) are
// applied in FP64 to the recombined value, which is split again.  Scratch
// holds one split complex (16 bytes) per point, like the FP64 path.
__device__ __forceinline__ CF cf_scale64(const CF &a, double2 m)  // split(a * m), product in FP64
{
    const double2 x = cf_to(a);
    return cf_from(x.x * m.x - x.y * m.y, x.x * m.y + x.y * m.x);
}
__device__ __forceinline__ CF cf_scale64c(const CF &a, double2 m)  // split(a * conj(m))
{
    const double2 x = cf_to(a);
    return cf_from(x.x * m.x + x.y * m.y, x.y * m.x - x.x * m.y);
}

__device__ __forceinline__ void tile_lds_ff(const Mp &p, const JobArgs &j, float4 *lds, const double2 *twl,
                                            const float4 *twf)
{
    const int lgN = j.lgN;
    const ll N = ll(1) << lgN;
    const double invN = 1.0 / (double)N;
    const Spec q = make_spec(p, j.h, j.beta, 0.0);
    const int tid = threadIdx.x;
    for (int t = tid; t < N; t += WG) st_cf(lds + t, cf_from(t < j.n_in ? tilt_in(j.src[t], j.beta, t, j.tc) : 0.0, 0.0));
    __syncthreads();
    lds_dif_ff(lds, lgN, 1, twf);
    for (ll f = tid; f <= N / 2; f += WG) {
        double cs, sn, sh;
        bin_trig_lds11(twl, f, lgN, cs, sn, sh);  // N <= 2048
        const double2 m = kernel_power(q, cs, sn, sh);
        const unsigned t1 = bitrev((unsigned)f, lgN), t2 = bitrev((unsigned)((N - f) & (N - 1)), lgN);
        st_cf(lds + t1, cf_scale64(ld_cf(lds + t1), m));
        if (t2 != t1) st_cf(lds + t2, cf_scale64c(ld_cf(lds + t2), m));
    }
    __syncthreads();
    lds_dit_inv_ff(lds, lgN, 1, twf);
    for (ll t = tid; t < j.n_out; t += WG) {
        const CF v = ld_cf(lds + j.out_off + t);
        j.dst[t] = tilt_out(((double)v.rh + (double)v.rl) * invN, j.beta, j.out_off + t, j.tc);
    }
    __syncthreads();
}

__device__ __forceinline__ void tile_col_fwd_ff(const JobArgs &j, int tile, float4 *lds, const double2 *__restrict__ tw,
                                                const float4 *twf)
{
    const int lgN = j.lgN, lg2 = LG_NLDS, lg1 = lgN - lg2;
    const ll N = ll(1) << lgN, N2 = ll(1) << lg2;
    const int N1 = 1 << lg1, C = NLDS >> lg1;
    const ll n20 = (ll)tile * C;
    const int tid = threadIdx.x;
    float4 *scr = (float4 *)j.scr;
    for (int t = tid; t < NLDS; t += WG) {
        const int c = t % C, n1 = t / C;
        const ll idx = (ll)n1 * N2 + n20 + c;
        st_cf(lds + c * N1 + n1, cf_from(idx < j.n_in ? tilt_in(j.src[idx], j.beta, idx, j.tc) : 0.0, 0.0));
    }
    __syncthreads();
    lds_dif_ff(lds, lg1, C, twf);
    for (int t = tid; t < NLDS; t += WG) {
        const int c = t % C, p1 = t / C;
        const ll k1 = bitrev(p1, lg1), n2 = n20 + c;
        const double2 w = twiddle_n((n2 * k1) & (N - 1), lgN);
        st_cf(scr + (ll)p1 * N2 + n2, cf_scale64(ld_cf(lds + c * N1 + p1), w));
    }
    __syncthreads();
}

__device__ __forceinline__ void tile_rows_ff(const Mp &p, const JobArgs &j, int tile, float4 *lds,
                                             const double2 *twl, const float4 *twf)
{
    const int lgN = j.lgN, lg2 = LG_NLDS, lg1 = lgN - lg2;
    const ll N2 = ll(1) << lg2;
    const Spec q = make_spec(p, j.h, j.beta, 0.0);
    const int tid = threadIdx.x;
    const int p1 = tile;
    const ll k1 = bitrev(p1, lg1);
    float4 *row = (float4 *)j.scr + (ll)p1 * N2;
    for (int t = tid; t < N2; t += WG) lds[t] = row[t];
    __syncthreads();
    lds_dif_ff(lds, lg2, 1, twf);
    double sr, cr;
    sincospi((double)(2 * k1) / (double)(ll(1) << lgN), &sr, &cr);
    const double2 r1 = make_double2(cr, -sr);
    sincospi((double)k1 / (double)(ll(1) << lgN), &sr, &cr);
    const double2 r2 = make_double2(cr, -sr);
    for (int k2 = tid; k2 < N2; k2 += WG) {  // natural bin order, as in tile_rows
        const int t = (int)bitrev(k2, lg2);
        double cs, sn, sh;
        bin_trig_rows(twl, r1, r2, k2, cs, sn, sh);
        st_cf(lds + t, cf_scale64(ld_cf(lds + t), kernel_power(q, cs, sn, sh)));
    }
    __syncthreads();
    lds_dit_inv_ff(lds, lg2, 1, twf);
    for (int t = tid; t < N2; t += WG) row[t] = lds[t];
    __syncthreads();
}

__device__ __forceinline__ void tile_col_inv_ff(const JobArgs &j, int tile, float4 *lds, const double2 *__restrict__ tw,
                                                const float4 *twf)
{
    const int lgN = j.lgN, lg2 = LG_NLDS, lg1 = lgN - lg2;
    const ll N = ll(1) << lgN, N2 = ll(1) << lg2;
    const int N1 = 1 << lg1, C = NLDS >> lg1;
    const double invN = 1.0 / (double)N;
    const ll n20 = (ll)tile * C;
    const int tid = threadIdx.x;
    const float4 *scr = (const float4 *)j.scr;
    for (int t = tid; t < NLDS; t += WG) {
        const int c = t % C, p1 = t / C;
        const ll k1 = bitrev(p1, lg1), n2 = n20 + c;
        const double2 w = twiddle_n((n2 * k1) & (N - 1), lgN);
        st_cf(lds + c * N1 + p1, cf_scale64c(ld_cf(scr + (ll)p1 * N2 + n2), w));
    }
    __syncthreads();
    lds_dit_inv_ff(lds, lg1, C, twf);
    for (int t = tid; t < NLDS; t += WG) {
        const int c = t % C, n1 = t / C;
        const ll idx = (ll)n1 * N2 + n20 + c;
        if (idx >= j.out_off && idx < j.out_off + j.n_out) {
            const CF v = ld_cf(lds + c * N1 + n1);
            j.dst[idx - j.out_off] = tilt_out(((double)v.rh + (double)v.rl) * invN, j.beta, idx, j.tc);
        }
    }
    __syncthreads();
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

// Direct stepping of a correlation whose input may exceed one wave's 1024
// cells: the output is cut into segments, each computed by direct_wave from
// its own input window (the segment plus the h-step dependency halo: span*h
// cells to the right for the lattices, h on each side for the centred BSM
// stencil).  Every output cell sees exactly the arithmetic of the unsplit
// computation.  Segments k = part, part + nparts, ... go to the caller.
__device__ __forceinline__ void direct_one(const Mp &p, const double *src, ll n_in, ll h, ll out_off, ll n_out,
                                           double *dst)
{
    if (n_in <= 128) direct_wave<2>(p, src, n_in, h, out_off, n_out, dst);
    else if (n_in <= 256) direct_wave<4>(p, src, n_in, h, out_off, n_out, dst);
    else if (n_in <= 512) direct_wave<8>(p, src, n_in, h, out_off, n_out, dst);
    else direct_wave<16>(p, src, n_in, h, out_off, n_out, dst);
}
__device__ __forceinline__ int direct_nseg(const Mp &p, ll n_in, ll h, ll n_out)
{
    const ll halo = (p.model == BINOMIAL) ? h : 2 * h;
    if (n_in <= 1024) return 1;
    const ll per = 1024 - halo;  // outputs per segment
    return (int)((n_out + per - 1) / per);
}
__device__ __forceinline__ void direct_part(const Mp &p, const double *src, ll n_in, ll h, ll out_off, ll n_out,
                                            double *dst, int part, int nparts)
{
    const int nseg = direct_nseg(p, n_in, h, n_out);
    if (nseg == 1) {
        if (part == 0) direct_one(p, src, n_in, h, out_off, n_out, dst);
        return;
    }
    const ll per = (n_out + nseg - 1) / nseg;
    for (int k = part; k < nseg; k += nparts) {
        const ll a = (ll)k * per;
        const ll b = (a + per < n_out) ? a + per : n_out;
        if (p.model == BSM) {
            // outputs a..b-1 are cells out_off+a .. out_off+b-1 of the input
            const ll lo = out_off + a - h, hi = out_off + b + h;  // window [lo, hi), lo >= 0
            const ll nin = (hi < n_in ? hi : n_in) - lo;
            direct_one(p, src + lo, nin, h, h, b - a, dst + a);
        } else {
            const ll span = (p.model == BINOMIAL) ? 1 : 2;
            const ll hi = b + span * h;
            const ll nin = (hi < n_in ? hi : n_in) - a;
            direct_one(p, src + a, nin, h, 0, b - a, dst + a);
        }
    }
}

__device__ __forceinline__ ll clk() { return (ll)__builtin_amdgcn_s_memtime(); }

// The kernel spectrum of an h-step correlation of N = 2^lgN <= 2^SPC_LG
// points, bins f = 0 .. N/2 (the rest is its mirror's conjugate), into out.
// Sub-trapezoids of one level share their heights, so a driver reuses these
// arrays across its private correlations (the spectrum cache in Ctx).
__device__ __forceinline__ void spec_fill(const Mp &p, ll h, int lgN, double2 *out, const double2 *twl,
                                          const double2 *__restrict__ tw)
{
    const Spec q = make_spec(p, h, 0.0, 0.0);
    const ll N = ll(1) << lgN;
    for (ll f = threadIdx.x; f <= N / 2; f += WG) {
        double cs, sn, sh;
        bin_trig_lds(twl, tw, f, lgN, cs, sn, sh);
        out[f] = kernel_power(q, cs, sn, sh);
    }
}

// One tile of a job, executed by the whole workgroup (control flow uniform).
template <int PREC>
__device__ __forceinline__ void run_tile(const Mp &p, const JobArgs &j, int ph, int t, double2 *lds,
                                         const double2 *__restrict__ tw, const double2 *twl, const float4 *twf,
                                         const double2 *spec = nullptr)
{
    if (j.kind == K_DIRECT) {
        direct_part(p, j.src, j.n_in, j.h, j.out_off, j.n_out, j.dst, threadIdx.x >> 6, WG / 64);
        __syncthreads();
    } else if (PREC) {
        float4 *l4 = (float4 *)lds;
        if (j.kind == K_LDS) tile_lds_ff(p, j, l4, twl, twf);
        else if (ph == 0) tile_col_fwd_ff(j, t, l4, tw, twf);
        else if (ph == 1) tile_rows_ff(p, j, t, l4, twl, twf);
        else tile_col_inv_ff(j, t, l4, tw, twf);
    } else if (j.kind == K_LDS) {
        tile_lds(p, j, lds, tw, twl, spec);
    } else if (ph == 0) {
        tile_col_fwd(j, t, lds, tw, twl);
    } else if (ph == 1) {
        tile_rows(p, j, t, lds, tw, twl, spec);
    } else {
        tile_col_inv(j, t, lds, tw, twl);
    }
}

// ------------------------------------------------------------ band walkers
// Executed by the 64 lanes of wave 0.  Lane l holds one cell of the current
// row; the neighbour a row step needs comes from the next lane by a DPP wave
// shift, and the cell beyond the band (an exercise cell) rides in as the
// shift's fill value.  Exercise values are carried per lane by one update per
// row and re-seeded with exp() every 64 rows.
//
// Boundary tracking uses the structure the paper proves: from one row to the
// next the last continuation cell either stays or moves one cell towards the
// root's side (Corollary 2.6, Theorem 4.2).  So each row only tests the ballot
// bit of the previous boundary cell: set -> the boundary stays, clear -> it
// drops by one.  This is the rule the oracle's last-red scan follows wherever
// the red cells are contiguous; the two can differ only where rounding makes a
// near-tie cell flip.  Per-row boundaries are collected (one row per lane, 64
// rows per store) only when the caller asks for them.

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

// One row step of a lattice band (TRI: trinomial).  Lane l holds columns
// c0+2l (A) and c0+2l+1 (B); eA, eB are their exercise values S u^{.} - K,
// advanced to the new row by e <- u e + K(u-1); f1 (f2) is the exercise value
// of column c0+128 (c0+129) in the row being read, the cells beyond the band
// that enter through the shift's fill.  rA, rB: whether the lane's new cells
// are red (continuation >= exercise, continuation finite).  GUARD = false is
// the fast form used by the count-based block check: the max of continuation
// and exercise value, which differs from the guarded rule only once a value
// has overflowed -- the block then ends with a non-finite cell and is walked
// again with GUARD = true.
template <bool TRI, bool GUARD>
__device__ __forceinline__ void lat_step(double &gA, double &gB, double &eA, double &eB, double &f1, double &f2,
                                         double u, double ku, double w0, double w1, double w2, bool &rA, bool &rB)
{
    // column c0+2l+2 (and c0+2l+3) is the next lane's A (B) cell; lane 63
    // receives the fills, and the next fills are computed from its shifted
    // registers
    const double nA = dpp_dn1(gA, f1);
    f1 = fma(nA, u, ku);
    double cA, cB;
    if (TRI) {
        const double nB = dpp_dn1(gB, f2);
        f2 = fma(nB, u, ku);
        cA = fma(w2, nA, fma(w1, gB, w0 * gA));
        cB = fma(w2, nB, fma(w1, nA, w0 * gB));
    } else {
        cA = fma(w1, gB, w0 * gA);
        cB = fma(w1, nA, w0 * gB);
    }
    eA = fma(eA, u, ku);
    eB = fma(eB, u, ku);
    if (!GUARD) {
        gA = vmax_f64(cA, eA);
        gB = vmax_f64(cB, eB);
        rA = cA >= eA;
        rB = cB >= eB;
        return;
    }
    // Definition 2.1 with the non-finite guard: c >= e and c finite (then e
    // is finite too).  A continuation value that overflowed marks an exercise
    // cell, whose value is its exercise value.
    rA = (cA >= eA) && (cA < INFINITY);
    rB = (cB >= eB) && (cB < INFINITY);
    gA = rA ? cA : eA;
    gB = rB ? cB : eB;
}

// Rows i0-1 .. i0-h of a lattice (binomial: row i has columns 0..i, cell j
// reads j and j+1; trinomial: columns 0..2i, cell j reads j, j+1, j+2) from
// row i0, whose red cells are [c0, b] (b - c0 + 1 <= BAND2); columns >= c0
// only, two per lane.  Writes the red cells of row i0-h to dst, the boundary
// of each row to bnd (may be NULL); returns the last red column of row i0-h.
// *v0 receives the final value of column c0.
//
// Rows go in blocks of up to 64.  The fast form of a block keeps, per cell,
// only the number of red rows and the last red row; the block is accepted if
// these show the structure of Corollary 2.6 / Theorem 4.2 -- each cell red in
// a prefix of the rows, the red cells of every row contiguous from c0, and the
// boundary dropping by at most one cell per row -- and every row of the block
// lies inside the lattice for all 128 cells.  Then row r's boundary is c0 - 1
// plus the number of cells red for more than r rows.  Otherwise (a near-tie
// cell, rows near the apex) the block is stepped again from its saved first
// row with the same arithmetic and each row's boundary follows from the
// previous one by the one-cell rule (the previous boundary cell red: it stays;
// green: it moves left by one), or, below an entirely red trinomial row, as
// the row's last red cell.
template <bool TRI>
__device__ __forceinline__ ll band_lat(Mp p, ll i0_, ll c0_, ll h_, ll b_, const double *src, double *dst,
                                       ll *bnd, double *v0)
{
    // indices fit in 32 bits (T <= 2^21): scalar 32-bit bookkeeping
    const int i0 = (int)uni(i0_), c0 = (int)uni(c0_), h = (int)uni(h_), b = (int)uni(b_);
    const int l = threadIdx.x & 63;
    const int jA = c0 + 2 * l, jB = jA + 1;
    const int cs = TRI ? 1 : 2;   // exercise exponent: S u^{cs j - i}
    const int wr = TRI ? 2 : 1;   // last column of row i: wr i
    const double S = p.S, K = p.K, a = p.a, w0 = p.w0, w1 = p.w1, w2 = TRI ? p.w2 : 0.0;
    const double u = exp(a);
    const double ku = K * (u - 1.0);
    double gA = (jA <= b) ? src[jA] : ((jA <= wr * i0) ? S * exp((double)(cs * jA - i0) * a) - K : 0.0);
    double gB = (jB <= b) ? src[jB] : ((jB <= wr * i0) ? S * exp((double)(cs * jB - i0) * a) - K : 0.0);
    int bc = b;
    // The carried exercise values e <- u e + K(u-1) amplify their rounding by
    // u per row: blocks (and re-seeding with exp) are cut to at most 4/a rows,
    // so that the amplification stays below e^4.  Every row length of a
    // practical lattice (a <= 1/16) keeps the full 64-row block.
    const int blk = (a * 64.0 <= 4.0) ? 64 : max(1, (int)(4.0 / a));
    for (int k0 = 0; k0 < h; k0 += blk) {
        const int nb = (h - k0) < blk ? (h - k0) : blk;
        const int itop = i0 - k0;  // row above the block
        const double eA0 = S * exp((double)(cs * jA - itop) * a) - K;
        const double eB0 = S * exp((double)(cs * jB - itop) * a) - K;
        const double f10 = S * exp((double)(cs * (c0 + BAND2) - itop) * a) - K;
        const double f20 = TRI ? fma(f10, u, ku) : 0.0;
        const int L0 = bc - c0;
        bool done = false;
        if (wr * (itop - nb) - c0 >= BAND2 - 1 && L0 >= 0 && L0 <= BAND2 - 1) {
            double ga = gA, gb = gB, ea = eA0, eb = eB0, f1 = f10, f2 = f20;
            int na = 0, nbb = 0, la = -1, lb = -1;
            bool rA, rB;
            if (nb == 64) {
#pragma unroll
                for (int r = 0; r < 64; ++r) {
                    lat_step<TRI, false>(ga, gb, ea, eb, f1, f2, u, ku, w0, w1, w2, rA, rB);
                    na += rA ? 1 : 0;
                    la = rA ? r : la;
                    nbb += rB ? 1 : 0;
                    lb = rB ? r : lb;
                }
            } else {
                for (int r = 0; r < nb; ++r) {
                    lat_step<TRI, false>(ga, gb, ea, eb, f1, f2, u, ku, w0, w1, w2, rA, rB);
                    na += rA ? 1 : 0;
                    la = rA ? r : la;
                    nbb += rB ? 1 : 0;
                    lb = rB ? r : lb;
                }
            }
            // counts of the next cells: cell 2l+1 is this lane's B, cell 2l+2
            // the next lane's A (cell 127 never needs one: it is at or beyond L0)
            const int nxtA = nbb;
            const int nxtB = __shfl_down(na, 1, 64);
            const int xA = 2 * l, xB = 2 * l + 1;
            const bool okA = ((na == 0) || (la == na - 1)) &&
                             ((xA > L0) ? (na == 0) : (xA == L0 || na > nxtA || (na == nb && nxtA == nb)));
            const bool okB = ((nbb == 0) || (lb == nbb - 1)) &&
                             ((xB > L0) ? (nbb == 0) : (xB == L0 || nbb > nxtB || (nbb == nb && nxtB == nb)));
            // a non-finite value (overflow) anywhere: the guarded walk below decides
            const bool finite = (ga < INFINITY) && (ea < INFINITY) && (gb < INFINITY) && (eb < INFINITY);
            if (__ballot(!(okA && okB && finite)) == 0ull) {
                gA = ga;
                gB = gb;
                bc = c0 - 1 + (int)__popcll(__ballot(na == nb)) + (int)__popcll(__ballot(nbb == nb));
                if (bnd) {
                    // lane r: row r's boundary, c0 - 1 plus the cells red for more than r rows
                    int q = c0 - 1;
                    for (int m = 0; 2 * m <= L0; ++m) {
                        q += (__builtin_amdgcn_readlane(na, m) > l) ? 1 : 0;
                        q += (__builtin_amdgcn_readlane(nbb, m) > l) ? 1 : 0;
                    }
                    if (l < nb) bnd[itop - 1 - l] = q;
                }
                done = true;
            }
        }
        if (!done) {
            double ea = eA0, eb = eB0, f1 = f10, f2 = f20;
            int q = 0;
            for (int r = 0; r < nb; ++r) {
                bool rA, rB;
                lat_step<TRI, true>(gA, gB, ea, eb, f1, f2, u, ku, w0, w1, w2, rA, rB);
                // cells beyond the row's last column are outside the lattice
                const int i = itop - 1 - r;
                const int lim = wr * i - c0;
                const unsigned long long mA = __ballot(rA) & row_mask(lim < 0 ? -1 : lim >> 1);
                const unsigned long long mB = __ballot(rB) & row_mask(lim < 1 ? -1 : (lim - 1) >> 1);
                if (TRI && bc >= wr * (i + 1)) {
                    // the row above was entirely red: this row's last red cell
                    int x = -1;
                    if (mB) x = 2 * (63 - (int)__clzll(mB)) + 1;
                    if (mA) x = max(x, 2 * (63 - (int)__clzll(mA)));
                    bc = c0 + x;
                } else {
                    const int lc = bc - c0;
                    if (lc >= 0 && lc < BAND2) bc -= ((((lc & 1) ? mB : mA) >> (lc >> 1)) & 1ull) ? 0 : 1;
                }
                q = (l == r) ? bc : q;
            }
            if (bnd && l < nb) bnd[itop - 1 - l] = q;
        }
    }
    if (jA <= bc) dst[jA] = gA;
    if (jB <= bc) dst[jB] = gB;
    if (v0 && l == 0) *v0 = gA;
    return bc;
}

// Band of a Bermudan binomial call (exercise on the rows i with (T - i) % d
// == 0, d = p.ex_every >= 2): rows i0-1 .. i0-h from the exercise row i0,
// whose red cells are [c0, b].  On the other rows every cell is a
// continuation cell (the linear stencil only).  The cells beyond the band,
// right of the boundary of the exercise row above, are exercise cells there,
// so on the rows below their values are the n-step linear stencil applied to
// exercise values: S u^{2j-i} rho_S^n - K rho_K^n (the forward identity of the
// lattice), with rho_S = w_up u + w_dn / u, rho_K = w_dn + w_up and n the rows
// since that exercise row.  The boundary of an exercise row is its last red
// cell (the ballot's highest lane); the other rows report their last column.
// Returns the boundary of row i0-h (an exercise row for trapezoid leaves).
__device__ __noinline__ ll band_bermudan(Mp p, ll i0_, ll c0_, ll h_, ll b_, const double *src, double *dst,
                                         ll *bnd, double *v0)
{
    const int i0 = (int)uni(i0_), c0 = (int)uni(c0_), h = (int)uni(h_), b = (int)uni(b_);
    const int T = (int)p.T, ev = p.ex_every;
    const int l = threadIdx.x & 63;
    const int j = c0 + l;
    const double S = p.S, K = p.K, a = p.a, w0 = p.w0, w1 = p.w1;
    const double u = exp(a);
    const double ku = K * (u - 1.0);
    const double lrs = log(w1 * u + w0 / u), lrk = log(w0 + w1);
    double g = (j <= b) ? src[j] : ((j <= i0) ? S * exp((double)(2 * j - i0) * a) - K : 0.0);
    double e = 0.0;
    // the fill: value of column c0 + 64 in the row being read
    double f1 = S * exp((double)(2 * (c0 + BAND) - i0) * a) - K;
    int bc = b;
    const int reseed = (a * 64.0 <= 4.0) ? 64 : max(1, (int)(4.0 / a));
    for (int k = 1; k <= h; ++k) {
        const int i = i0 - k;
        if ((k - 1) % reseed == 0) e = S * exp((double)(2 * j - (i + 1)) * a) - K;  // row i+1, then advanced
        const double g1 = dpp_dn1(g, f1);
        const double c = fma(w1, g1, w0 * g);
        e = fma(e, u, ku);
        const int n = (T - i) % ev;  // rows since the exercise row above (0: row i exercises)
        if (n == 0) {
            const bool red = (c >= e) && (c < INFINITY);
            g = red ? c : e;
            const unsigned long long m = __ballot(red) & row_mask(i - c0);
            bc = m ? c0 + 63 - (int)__clzll(m) : c0 - 1;
            if (bnd && l == 0) bnd[i] = bc;
        } else {
            g = c;
            if (bnd && l == 0) bnd[i] = i;
        }
        f1 = S * exp((double)(2 * (c0 + BAND) - i) * a + (double)n * lrs) - K * exp((double)n * lrk);
    }
    if (j <= bc) dst[j] = g;
    if (v0 && l == 0) *v0 = g;
    return bc;
}

__device__ __forceinline__ ll band_bin(Mp p, ll i0, ll c0, ll h, ll b, const double *src, double *dst, ll *bnd,
                                       double *v0)
{
    if (p.ex_every > 1) return band_bermudan(p, i0, c0, h, b, src, dst, bnd, v0);
    return band_lat<false>(p, i0, c0, h, b, src, dst, bnd, v0);
}
__device__ __forceinline__ ll band_tri(Mp p, ll i0, ll c0, ll h, ll b, const double *src, double *dst, ll *bnd,
                                       double *v0)
{
    return band_lat<true>(p, i0, c0, h, b, src, dst, bnd, v0);
}

// One step of the BSM band, two cells per lane: lane l holds positions 2l (A)
// and 2l+1 (B) of the band, which moves one cell to the left per step, so the
// new A cell needs old positions 2l-2, 2l-1, 2l (the previous lane's A and B,
// its own A) and the new B cell old positions 2l-1, 2l, 2l+1; lane 0 takes
// exercise values for the cells left of the band.  xA is e^{s} of the lane's
// A cell (its new B cell is its old A cell).  rA, rB: whether the new cells
// are continuation (not exercise).
__device__ __forceinline__ void bsm_step(double &vA, double &vB, double &xA, double ud, double w0, double w1,
                                         double w2, bool &rA, bool &rB)
{
    const double xB = xA;
    xA *= ud;
    const double gA = 1.0 - xA, gB = 1.0 - xB;
    const double pA = dpp_up1(vA, 1.0 - xA * ud);  // old position 2l-2 (lane 0: the cell left of the new A)
    const double pB = dpp_up1(vB, gA);             // old position 2l-1 (lane 0: the new A cell itself)
    const double cA = fma(w2, vA, fma(w1, pB, w0 * pA));
    const double cB = fma(w2, vB, fma(w1, vA, w0 * pB));
    vA = vmax_f64(cA, gA);
    vB = vmax_f64(cB, gB);
    rA = !(gA > cA);
    rB = !(gB > cB);
}

// BSM put: steps n0+1 .. n0+h from step n0, whose exercise cells are k <= f
// and whose continuation cells [f+1, R0] are read from src (absolute k).  The
// band (128 cells, two per lane) has its right edge at R0 and moves left one
// cell per step (the dependency cone); its left part stays inside the
// exercise region (needs R0 - f <= 126).  Writes the red cells of step n0+h,
// up to R0-h, to dst and returns the last exercise offset of step n0+h.  *vr
// receives the value of the rightmost cell (the apex when R0 - h = 0).  Here
// the boundary is the last exercise (green) cell; it stays or moves one cell
// left per step (Theorem 4.2), so in band positions (which move left with the
// band) the exercise prefix grows by 0 or 1 position per step.
__device__ __forceinline__ ll band_bsm(Mp p, ll n0_, ll f_, ll h_, ll R0_, const double *src, double *dst,
                                       ll *bnd, double *vr)
{
    // offsets k lie in [-2T-1, T+1]: 32-bit scalar bookkeeping
    const int n0 = (int)uni(n0_), f = (int)uni(f_), h = (int)uni(h_), R0 = (int)uni(R0_);
    const int l = threadIdx.x & 63;
    const int T = (int)p.T;
    const double w0 = p.w0, w1 = p.w1, w2 = p.w2, s0 = p.s0, ds = p.a;
    const double ud = exp(-ds);  // e^{-ds}: one cell to the left
    int base = R0 - (BAND2 - 1);
    const int kA = base + 2 * l, kB = kA + 1;
    double vA = (kA <= f) ? 1.0 - exp(s0 + (double)kA * ds) : src[kA];
    double vB = (kB <= f) ? 1.0 - exp(s0 + (double)kB * ds) : src[kB];
    int fc = f;
    for (int t0 = 0; t0 < h; t0 += 64) {
        const int nb = (h - t0) < 64 ? (h - t0) : 64;
        const int base0 = base;                                     // band base before the block
        const double x0 = exp(s0 + (double)(base0 + 2 * l) * ds);  // e^{s} of the lane's A cell before the block
        // Fast form (as band_lat): per cell the number of continuation rows and
        // the last one.  Row r of the block has position 0 at cell base0 - 1 - r,
        // so the exercise positions (0 .. G_r - 1) grow by 0 or 1 per row.
        bool done = false;
        {
            double va = vA, vb = vB, x = x0;
            int na = 0, nbb = 0, la = -1, lb = -1;
            bool rA, rB;
            if (nb == 64) {
#pragma unroll
                for (int r = 0; r < 64; ++r) {
                    bsm_step(va, vb, x, ud, w0, w1, w2, rA, rB);
                    na += rA ? 1 : 0;
                    la = rA ? r : la;
                    nbb += rB ? 1 : 0;
                    lb = rB ? r : lb;
                }
            } else {
                for (int r = 0; r < nb; ++r) {
                    bsm_step(va, vb, x, ud, w0, w1, w2, rA, rB);
                    na += rA ? 1 : 0;
                    la = rA ? r : la;
                    nbb += rB ? 1 : 0;
                    lb = rB ? r : lb;
                }
            }
            // counts of the next positions: 2l+1 is this lane's B, 2l+2 the next lane's A
            const int nxtA = nbb;
            const int nxtB = __shfl_down(na, 1, 64);
            const bool okA = ((na == 0) || (la == na - 1)) &&
                             (na < nxtA || (na == nxtA && (na == 0 || na == nb)));
            const bool okB = ((nbb == 0) || (lb == nbb - 1)) &&
                             (l == 63 || nbb < nxtB || (nbb == nxtB && (nbb == 0 || nbb == nb)));
            const int g0 = (int)__popcll(__ballot(na == 0)) + (int)__popcll(__ballot(nbb == 0));  // exercise positions of the first row
            const int gin = fc - base0 + 1;
            if (__ballot(!(okA && okB)) == 0ull && g0 >= 1 && (g0 == gin || g0 == gin + 1)) {
                vA = va;
                vB = vb;
                const int glast = BAND2 - (int)__popcll(__ballot(na == nb)) - (int)__popcll(__ballot(nbb == nb));
                fc = base0 - nb + glast - 1;
                if (bnd) {
                    // lane r: row r's last exercise cell
                    int q = base0 - 1 - l - 1;
                    for (int m = 0; m < 64; ++m) {
                        q += (__builtin_amdgcn_readlane(na, m) <= l) ? 1 : 0;
                        q += (__builtin_amdgcn_readlane(nbb, m) <= l) ? 1 : 0;
                    }
                    if (l < nb) {
                        const int n = n0 + t0 + 1 + l;
                        bnd[n] = (q < -(T - n)) ? BSM_NONE : (ll)(q > T - n ? T - n : q);
                    }
                }
                done = true;
            }
        }
        if (!done) {
            // the one-cell rule row by row: the previous boundary cell still
            // exercise, it stays; continuation, the boundary moves left by one
            double x = x0;
            int q = 0;
            for (int r = 0; r < nb; ++r) {
                bool rA, rB;
                bsm_step(vA, vB, x, ud, w0, w1, w2, rA, rB);
                const unsigned long long mA = __ballot(!rA), mB = __ballot(!rB);  // exercise positions
                const int pos = fc - (base0 - 1 - r);  // the previous boundary cell's position in this row
                if (pos >= 0 && pos < BAND2) fc -= ((((pos & 1) ? mB : mA) >> (pos >> 1)) & 1ull) ? 0 : 1;
                q = (l == r) ? fc : q;
            }
            if (bnd && l < nb) {
                const int n = n0 + t0 + 1 + l;
                bnd[n] = (q < -(T - n)) ? BSM_NONE : (ll)(q > T - n ? T - n : q);
            }
        }
        base -= nb;
    }
    const int ka = base + 2 * l, kb = ka + 1;
    if (ka > fc && ka <= R0 - h) dst[ka] = vA;
    if (kb > fc && kb <= R0 - h) dst[kb] = vB;
    if (vr && l == 63) *vr = vB;
    return fc;
}

// ---------------------------------------------------------------- work pool
// The solve kernel is persistent.  Each workgroup claims the next option
// (descriptors are sorted by decreasing cost) and drives it; once no option is
// left it becomes a helper.  A driver publishes its correlations as jobs in its
// own slots (slot 0: top level, slot s+1: recursion depth s); any workgroup
// may claim a tile of a published job with one atomic add on the job's control
// word.  A driver that needs a job's result claims the job's remaining tiles
// itself, so a wait only ever depends on tiles that running workgroups have
// claimed: the scheme cannot deadlock, whatever the number of resident
// workgroups.  Every wait is bounded by a deadline as well; past it the launch
// aborts and the options still in flight price NaN.
//
// Memory ordering (agent scope): a publisher's row data and job arguments are
// released before the control word is stored; a claimer acquires after its
// atomic add; a tile's writes are released before its completion is counted;
// the workgroup that completes a phase opens the next one, or marks the job
// done, with a release store, and the driver acquires before reading results.
struct Job {
    unsigned long long ctl;  // gen:16 | phase:8 | claimed:20 | total:20
    unsigned done[3];        // completed tiles per phase
    int pad;
    JobArgs a;
};
static_assert(sizeof(Job) <= JOB_BYTES, "job slot");

#define PH_DONE 0xFFu
#define SLOT_TOP 0
#define AGENT __HIP_MEMORY_SCOPE_AGENT

__device__ __forceinline__ unsigned long long mkctl(unsigned gen, unsigned ph, unsigned claimed, unsigned total)
{
    return ((unsigned long long)(gen & 0xFFFFu) << 48) | ((unsigned long long)ph << 40) |
           ((unsigned long long)claimed << 20) | (unsigned long long)total;
}
__device__ __forceinline__ unsigned ctl_ph(unsigned long long c) { return (unsigned)(c >> 40) & 0xFFu; }
__device__ __forceinline__ unsigned ctl_claimed(unsigned long long c) { return (unsigned)(c >> 20) & 0xFFFFFu; }
__device__ __forceinline__ unsigned ctl_total(unsigned long long c) { return (unsigned)c & 0xFFFFFu; }
__device__ __forceinline__ unsigned ctl_gen(unsigned long long c) { return (unsigned)(c >> 48); }

struct Pool {
    PoolHdr *hdr;
    unsigned long long *summary;  // bit w: workgroup w has a flagged slot (maintained loosely)
    unsigned long long *bits;     // [n_wg]: bit s of word w = slot s of workgroup w has claimable tiles
    Job *jobs;                    // [n_wg * JPW]
    int *drivers;                 // [MAX_WG]: workgroup driving option o (-1 not yet claimed)
    int n_wg;
};

// Shared control words are only ever read with atomic read-modify-writes:
// those are performed at the device's coherence point, whereas a plain or
// relaxed load may keep returning a line cached before another XCD wrote it.
__device__ __forceinline__ unsigned long long rmw_read(unsigned long long *p)
{
    return __hip_atomic_fetch_or(p, 0ull, __ATOMIC_RELAXED, AGENT);
}
// A workgroup barrier orders global stores only within the workgroup.  Where
// one lane then releases them to other workgroups (publishing a job,
// counting a finished tile), every wave first waits until its own stores
// have completed, so that the lane's agent-scope release covers the stores
// of the whole workgroup.
__device__ __forceinline__ void sync_stores()
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
}
__device__ __forceinline__ void fence_acq() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ ll now_ticks() { return (ll)__builtin_amdgcn_s_memrealtime(); }
__device__ __forceinline__ bool aborted(const Pool &pl) { return (rmw_read((unsigned long long *)&pl.hdr->status) >> 32) != 0ull; }
__device__ __forceinline__ void set_abort(const Pool &pl)
{
    __hip_atomic_fetch_or((unsigned long long *)&pl.hdr->status, 1ull << 32, __ATOMIC_RELAXED, AGENT);
}
// Abort the launch and, if this is the first cause, record it (aop_pool_abort_info).
__device__ __forceinline__ void note_abort(const Pool &pl, ll reason, ll i1, ll i2, ll i3, ll i4, ll i5, ll i6)
{
    unsigned long long *w = (unsigned long long *)pl.hdr->abort_info;
    unsigned long long expect = 0ull;
    if (__hip_atomic_compare_exchange_strong(w, &expect, (unsigned long long)reason, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             AGENT)) {
        const ll v[6] = {i1, i2, i3, i4, i5, i6};
        for (int k = 0; k < 6; ++k) __hip_atomic_exchange(w + 1 + k, (unsigned long long)v[k], __ATOMIC_RELAXED, AGENT);
    }
    set_abort(pl);
}

// The summary bit of workgroup w may be stale in either direction; a helper
// that finds it set over an empty word clears it, and whoever clears it
// re-checks the word afterwards, so a set word never stays unannounced.
__device__ __forceinline__ void summary_clear_recheck(const Pool &pl, int w)
{
    __hip_atomic_fetch_and(pl.summary + (w >> 6), ~(1ull << (w & 63)), __ATOMIC_SEQ_CST, AGENT);
    if (__hip_atomic_fetch_or(pl.bits + w, 0ull, __ATOMIC_SEQ_CST, AGENT))
        __hip_atomic_fetch_or(pl.summary + (w >> 6), 1ull << (w & 63), __ATOMIC_RELAXED, AGENT);
}
__device__ __forceinline__ void flag_slot(const Pool &pl, int ji)
{
    const int w = ji / JPW;
    const unsigned long long old = __hip_atomic_fetch_or(pl.bits + w, 1ull << (ji % JPW), __ATOMIC_RELAXED, AGENT);
    if (old == 0ull) __hip_atomic_fetch_or(pl.summary + (w >> 6), 1ull << (w & 63), __ATOMIC_RELAXED, AGENT);
}
__device__ __forceinline__ void unflag_slot(const Pool &pl, int ji)
{
    const int w = ji / JPW;
    const unsigned long long bit = 1ull << (ji % JPW);
    const unsigned long long old = __hip_atomic_fetch_and(pl.bits + w, ~bit, __ATOMIC_RELAXED, AGENT);
    if ((old & ~bit) == 0ull) summary_clear_recheck(pl, w);
}

// Claim one tile of job ji (one lane).  True with *ph, *t set if the add
// landed on an open phase with an unclaimed tile; the lane that takes the last
// tile of a phase unflags the slot.
__device__ __forceinline__ bool claim_tile(const Pool &pl, int ji, int *ph, int *t)
{
    Job *jb = pl.jobs + ji;
    const unsigned long long c = __hip_atomic_fetch_add(&jb->ctl, 1ull << 20, __ATOMIC_RELAXED, AGENT);
    const unsigned p = ctl_ph(c), k = ctl_claimed(c), tot = ctl_total(c);
    if (p >= 3 || k >= tot) return false;
    if (k + 1 == tot) unflag_slot(pl, ji);
    fence_acq();
    *ph = (int)p;
    *t = (int)k;
    return true;
}

// Count a finished tile (one lane, after the whole workgroup's writes) of a
// job with nph phases of nt tiles; the lane that completes a phase opens the
// next one or marks the job done.
__device__ __forceinline__ void complete_tile(const Pool &pl, int ji, int ph, int nt, int nph)
{
    Job *jb = pl.jobs + ji;
    const unsigned d = __hip_atomic_fetch_add(&jb->done[ph], 1u, __ATOMIC_ACQ_REL, AGENT);
    if (d + 1 != (unsigned)nt) return;
    const unsigned gen = ctl_gen(rmw_read(&jb->ctl));
    if (ph + 1 < nph) {
        __hip_atomic_exchange(&jb->ctl, mkctl(gen, ph + 1, 0, nt), __ATOMIC_RELEASE, AGENT);
        flag_slot(pl, ji);
    } else {
        __hip_atomic_exchange(&jb->ctl, mkctl(gen, PH_DONE, 0, 0), __ATOMIC_RELEASE, AGENT);
    }
}

// Copy a job's arguments into LDS (lanes 0..11 of wave 0, after the claim's
// acquire).  A slot's arguments are rewritten for every job published in it,
// so this workgroup's L2 may still hold the previous job's: like the control
// words they are read with atomic read-modify-writes (and written with atomic
// exchanges), which are performed at the device's coherence point.
__device__ __forceinline__ void fetch_args(const Pool &pl, int ji, JobArgs *sh)
{
    const int l = threadIdx.x;
    if (l < (int)(sizeof(JobArgs) / 8)) {
        unsigned long long *w = (unsigned long long *)&pl.jobs[ji].a;
        ((unsigned long long *)sh)[l] = rmw_read(w + l);
    }
}

// Per-workgroup LDS state shared by the driver and helper roles.
// Queue through which the wave that solves a small trapezoid hands its
// direct-stepping correlations to the workgroup's other waves (all in LDS).
// A frame has at most one outstanding correlation, kept in the job slot of
// its stack depth until the frame has waited for it.  A correlation longer
// than one wave's segment is queued as one ticket per output segment, so
// that the waves step its segments side by side; tickets (numbered in push
// order) name a slot and a part, and a slot's count of parts left reaches
// zero when its job is done.
#define WQ 16   // job slots = deepest stack
#define WQT 64  // ticket ring: at most WQ frames, few of them longer than one segment
struct WJob {
    const double *src;
    double *dst;
    ll n_in, h, out_off, n_out;
};
struct WQueue {
    WJob job[WQ];
    int left[WQ];     // parts of the slot's job not yet finished
    int ticket[WQT];  // ticket k: slot | part << 8 | parts << 16, at k % WQT
    int head;         // next ticket to claim
    int tail;         // tickets issued
    int quit;         // the pushing wave has finished
    int pad;
};

struct Shared {
    WQueue wq;
    int msg, ji, opt, pad;
    ll spk[SPC_E];  // spectrum cache keys (h << 8 | lgN), -1 empty
    int late, pad4[3];  // most of the launch's options are done: publish more (Tune::late_pub_lg)
    int spn, spx, spf, pad3;  // entries handed out; lookup result: entry, fill needed
    int spin[SPC_E];          // published jobs reading each spectrum-cache entry (not replaced while > 0)
    int sppub[JPW];           // cache entry read by each slot's published job, -1 none
    JobArgs args;          // arguments of the tile a helper claimed
    JobArgs jargs[JPW];    // arguments of each slot's pending job (driver)
    int pub[JPW];          // slot state: 0 idle, 1 published job pending, 2 private job pending
    unsigned gen[JPW];     // generation of the slot's last published job
};

// A helper: claim tiles of any published job until every option is done.
// A claimed job's arguments must describe ranges inside its option's own
// workspace area (rows, arena, FFT scratch); anything else is refused.
__device__ __forceinline__ bool args_ok(const Desc *__restrict__ descs, ll n, const char *ws, const JobArgs &a, int ph,
                                        int tile, int prec)
{
    if (a.desc < 0 || a.desc >= n || a.kind < K_DIRECT || a.kind > K_4STEP || a.lgN < 1 || a.lgN > LG_TW ||
        ph < 0 || ph >= a.nph || tile < 0 || tile >= a.ntile || a.n_in < 1 || a.n_out < 1 || a.n_in > (ll(1) << a.lgN) ||
        a.prec < 0 || a.prec > 1 || (a.kind != K_DIRECT && a.prec != prec) || a.radix < 2 || a.radix > 3 ||
        a.cached < 0 || a.cached > 1 || (a.cached && (a.kind != K_LDS || a.lgN > SPC_LG)))
        return false;
    const Desc d = descs[a.desc];
    if (d.model < 0) return false;
    const char *lo = ws + d.ws_off;
    const char *hi = lo + 8 * (2 * d.row_len + d.arena_len) + 16 * d.scr_len;
    const char *s0 = (const char *)a.src, *s1 = (const char *)(a.src + a.n_in);
    const char *d0 = (const char *)a.dst, *d1 = (const char *)(a.dst + a.n_out);
    if (s0 < lo || s1 > hi || d0 < lo || d1 > hi) return false;
    if (a.kind == K_LDS && a.lgN > lds_lg(prec)) return false;  // must fit the LDS buffer
    if (a.cached) {  // a spectrum-cache entry: after the FFT scratch
        const char *c0 = (const char *)a.scr, *c1 = (const char *)(a.scr + ((ll(1) << a.lgN) / 2 + 1));
        if (c0 < hi || c1 > hi + 16 * SPC_E * spc_entry(d.nfft)) return false;
    }
    if (a.kind == K_4STEP) {
        const char *c0 = (const char *)a.scr, *c1 = (const char *)(a.scr + (ll(1) << a.lgN));
        if (c0 < lo || c1 > hi || a.lgN <= LG_NLDS) return false;  // N1 >= 2 row tiles
    }
    return true;
}

// A helper leaves once every option is done, the launch aborted, or it has
// found nothing to claim for `idle_ticks` (helpers are never needed for
// progress: drivers finish their own jobs).
template <int PREC>
__device__ void helper_loop(const Pool &pl, ll n, const Desc *__restrict__ descs, const char *ws, Shared *sh,
                            double2 *lds, const double2 *__restrict__ tw, const double2 *twl, const float4 *twf,
                            ll idle_ticks)
{
    ll last_work = now_ticks();
    const int tid = threadIdx.x;
    const int l = tid & 63;
    const int nsum = (pl.n_wg + 63) >> 6;
    const ll t_start = clk();
    ll busy = 0, tiles = 0;
    unsigned rot = blockIdx.x * 37u;
    // Home driver: the helpers share the drivers out evenly -- the k-th
    // workgroup to enter this loop serves option k mod n first -- so that
    // every option keeps the same number of helpers of its own instead of
    // whatever the scan finds; any job may still be claimed.
    int home = -1, home_tries = 0;
    const int n_home = (int)(n < MAX_WG ? n : MAX_WG);
    int rank = 0;
    if (tid == 0) rank = (int)__hip_atomic_fetch_add(&pl.hdr->n_helpers, (int64_t)1, __ATOMIC_RELAXED, AGENT);
    rank = __builtin_amdgcn_readfirstlane(rank);
    const int home_opt = n_home > 0 ? rank % n_home : 0;
    for (;;) {
        if (tid < 64) {
            int msg = 0, ji = -1;  // 0 nothing, 1 tile, 2 exit
            if (home < 0 && home_tries < 64) {
                ++home_tries;
                int hd = -1;
                if (l == 0) hd = __hip_atomic_fetch_add(pl.drivers + home_opt, 0, __ATOMIC_RELAXED, AGENT);
                hd = __builtin_amdgcn_readfirstlane(hd);
                if (hd >= 0 && hd != (int)blockIdx.x && hd < pl.n_wg) home = hd;
            }
            unsigned long long st = 0ull, sw = 0ull;
            if (l == 0) st = rmw_read((unsigned long long *)&pl.hdr->status);
            if (l < nsum) sw = rmw_read(pl.summary + l);
            st = ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)(st >> 32), 0) << 32) |
                 (unsigned)__builtin_amdgcn_readlane((int)(unsigned)st, 0);
            if ((ll)(st & 0xffffffffull) >= n || (st >> 32) || now_ticks() - last_work > idle_ticks) {
                msg = 2;
            } else {
                if (home >= 0) {
                    int ok = 0, ph = 0, t = 0, cj = -1;
                    if (l == 0) {
                        const unsigned long long bw = rmw_read(pl.bits + home);
                        if (bw) {
                            cj = home * JPW + (63 - (int)__clzll(bw));  // deepest slot first
                            ok = claim_tile(pl, cj, &ph, &t);
                        }
                    }
                    if (__builtin_amdgcn_readfirstlane(ok)) {
                        msg = 1 | (__builtin_amdgcn_readfirstlane(ph) << 4) | (__builtin_amdgcn_readfirstlane(t) << 8);
                        ji = __builtin_amdgcn_readfirstlane(cj);
                    }
                }
                const unsigned long long m = msg ? 0ull : __ballot(sw != 0ull);
                if (m) {
                    // a workgroup with claimable work: rotate over summary words and bits
                    const int r = (int)(rot & 63u);
                    const unsigned long long rm = r ? ((m >> r) | (m << (64 - r))) : m;
                    const int lane = (__ffsll((long long)rm) - 1 + r) & 63;
                    int ok = 0, ph = 0, t = 0, cj = -1;
                    if (l == lane) {
                        const int r2 = (int)((rot >> 6) & 63u);
                        const unsigned long long sr = r2 ? ((sw >> r2) | (sw << (64 - r2))) : sw;
                        const int w = lane * 64 + ((__ffsll((long long)sr) - 1 + r2) & 63);
                        const unsigned long long bw = (w < pl.n_wg) ? rmw_read(pl.bits + w) : 0ull;
                        if (bw == 0ull) {
                            if (w < pl.n_wg) summary_clear_recheck(pl, w);
                        } else {
                            cj = w * JPW + (63 - (int)__clzll(bw));  // deepest slot first
                            ok = claim_tile(pl, cj, &ph, &t);
                        }
                    }
                    ok = __builtin_amdgcn_readlane(ok, lane);
                    if (ok) {
                        msg = 1 | (__builtin_amdgcn_readlane(ph, lane) << 4) | (__builtin_amdgcn_readlane(t, lane) << 8);
                        ji = __builtin_amdgcn_readlane(cj, lane);
                    }
                }
                rot += 65u;
                if (msg == 0) __builtin_amdgcn_s_sleep(2);
            }
            if ((msg & 15) == 1) fetch_args(pl, ji, &sh->args);
            if (l == 0) {
                sh->msg = msg;
                sh->ji = ji;
            }
        }
        __syncthreads();
        const int msg = __builtin_amdgcn_readfirstlane(sh->msg);
        const int ji = __builtin_amdgcn_readfirstlane(sh->ji);
        const JobArgs a = uni_args(sh->args);
        __syncthreads();
        if ((msg & 15) == 2) break;
        if ((msg & 15) != 1) continue;
        const ll t0 = clk();
        const int ph = (msg >> 4) & 15, tile = msg >> 8;
        if (args_ok(descs, n, ws, a, ph, tile, PREC)) {
            const Mp p = make_mp(descs[a.desc]);
            run_tile<PREC>(p, a, ph, tile, lds, tw, twl, twf,
                           (a.kind == K_LDS && a.cached) ? (const double2 *)a.scr : nullptr);
        } else if (tid == 0) {
            note_abort(pl, 1, ji, ((ll)ph << 32) | tile,
                       ((ll)a.kind << 48) | ((ll)a.nph << 40) | ((ll)a.lgN << 32) | (ll)(unsigned)a.ntile,
                       ((ll)a.desc << 32) | (ll)(unsigned)a.n_in, a.n_out, (ll)rmw_read(&pl.jobs[ji].ctl));
        }
        sync_stores();
        if (tid == 0) complete_tile(pl, ji, ph, a.ntile, a.nph);
        busy += clk() - t0;
        ++tiles;
        last_work = now_ticks();
    }
    if (tid == 0) {
        __hip_atomic_fetch_add(&pl.hdr->helper_tiles, tiles, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_fetch_add(&pl.hdr->helper_busy, busy, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_fetch_add(&pl.hdr->helper_idle, clk() - t_start - busy, __ATOMIC_RELAXED, AGENT);
    }
}

// ---------------------------------------------------------- the recursion
struct Frame {
    ll r0;    // row i0 (lattices) / step n (BSM)
    ll c0;    // first red column (lattices) / boundary f (BSM)
    ll h;     // trapezoid height
    ll b;     // last red column of row r0 (lattices)
    ll aoff;  // arena offset (doubles) of this frame's middle-row buffer
    ll soff;  // FFT scratch offset (complex) of this frame's correlation
    double *src, *dst, *mid;
    int stage, pad;
};

struct Ctx {
    Mp p;
    int desc;         // descriptor index of the option
    Stats *st;        // work counters in LDS (updated by lane 0 only)
    double *lo, *hi;  // this option's workspace (doubles) for range checks
    double *arena;
    ll arena_len;
    double2 *scr;
    ll scr_len;
    double2 *spc;  // spectrum cache: SPC_E entries of spc_ent complex values
    ll spc_ent;
    double2 *lds;
    const double2 *tw;
    const double2 *twl;
    const float4 *twf;
    int prec;  // 0 FP64, 1 split-FP32 FFT correlations
    ll *bnd;
    Pool pl;
    Tune tn;
    Shared *sh;
    int *err_sh;
};

__device__ __forceinline__ bool in_ws(const Ctx &cx, const double *p, ll first, ll last)
{
    if (last < first) return true;
    return (p + first >= cx.lo) && (p + last < cx.hi);
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

__device__ __forceinline__ void set_err(const Ctx &cx, int e)
{
    if (threadIdx.x == 0 && *cx.err_sh == 0) *cx.err_sh = e;
}

// The cached kernel spectrum of an h-step correlation of 2^lgN points (see below).
__device__ __forceinline__ const double2 *spec_get(const Ctx &cx, ll h, int lgN, bool pin = false);

// Correlate src[0..n_in) with the h-step kernel and write the window
// [out_off, out_off + n_out) to dst (see the job description above), as the
// pending job of slot `slot`, using the FFT scratch from offset soff.  Large
// jobs are published to the pool; the others stay private to the driver.
// Either way the work is done (or finished) by conv_wait.  Returns the scratch
// (complex elements) the job holds until then.
template <int PREC>
__device__ __forceinline__ ll conv_submit(const Ctx &cx, int slot, ll soff, const double *src, ll n_in, ll h,
                                          ll out_off, ll n_out, double *dst, double beta = 0.0, double tc = 0.0,
                                          bool stage = false)
{
    if (n_out <= 0) return 0;
    count_conv(cx.st, n_in, n_out);
    JobArgs a;
    a.src = src;
    a.dst = dst;
    a.n_in = n_in;
    a.h = h;
    a.out_off = out_off;
    a.n_out = n_out;
    a.beta = beta;
    a.tc = tc;
    a.desc = cx.desc;
    int lgN = ceil_log2(n_in);
    if (lgN < 1) lgN = 1;
    a.lgN = lgN;
    const bool direct = beta == 0.0 && h <= cx.tn.direct_max_h && n_in <= cx.tn.direct_max_n;
    // FP64 transforms of up to 2^lds_lg64 points (11 or 12, tuned) run whole in LDS
    a.kind = direct ? K_DIRECT : (lgN <= (PREC ? LG_NLDS : cx.tn.lds_lg64) ? K_LDS : K_4STEP);
    a.prec = direct ? 0 : PREC;  // direct stepping is always FP64
    a.radix = cx.tn.radix;
    a.cached = 0;
    a.nph = a.kind == K_4STEP ? 3 : 1;
    a.ntile = a.kind == K_4STEP ? (1 << (lgN - LG_NLDS)) : 1;
    const ll need = a.kind == K_4STEP ? (ll(1) << lgN) : 0;
    a.scr = cx.scr + soff;
    if (soff + need > cx.scr_len || lgN > LG_TW || slot >= JPW) {
        set_err(cx, DEV_ARENA);
        return 0;
    }
    // late in the launch most workgroups are idle helpers and fences are
    // cheap: the drivers still running publish smaller correlations
    const int thr = (cx.tn.late_pub_lg > 0 && cx.sh->late) ? cx.tn.late_pub_lg : cx.tn.pub_min_lg;
    const bool publish = cx.pl.n_wg > 1 && (direct ? cx.tn.pub_direct != 0 : lgN >= thr);
    // A published whole-LDS job of the FP64 path takes its kernel spectrum from
    // the driver's cache (filled here on a miss), so that the tile reads it
    // instead of evaluating it; the entry stays pinned until the job is done.
    if (PREC == 0 && publish && a.kind == K_LDS && beta == 0.0 && lgN <= SPC_LG) {
        const double2 *e = spec_get(cx, h, lgN, true);
        if (e) {
            a.scr = (double2 *)e;
            a.cached = 1;
            if (threadIdx.x == 0) cx.sh->sppub[slot] = cx.sh->spx;
        }
    }
    if (publish) sync_stores();  // the workgroup's writes of the input row precede the release below
    // A private FP64 whole-LDS job of up to 2048 points whose frame next
    // solves a wave-level sub-trapezoid (which uses no FFT buffer) starts
    // loading its input now, straight from global memory into the staging
    // area of the LDS buffer, so that the loads complete while the
    // sub-trapezoid is solved (pairs of doubles; an odd last element is read
    // by the tile).
    if (PREC == 0 && stage && !publish && a.kind == K_LDS && beta == 0.0 && lgN <= LG_NLDS) {
        __syncthreads();  // the input row's writes by this workgroup precede the loads
        double *stg = (double *)(cx.lds + STG_OFF);
        const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
        const ll pairs = n_in >> 1;
        for (int k = 0; k * WG < pairs; ++k) {
            const ll pr = (ll)k * WG + w * 64 + l;  // pair of this lane
            if (pr < pairs)
                __builtin_amdgcn_global_load_lds((const void *)(src + 2 * pr),
                                                 (void __attribute__((address_space(3))) *)(stg + 2 * ((ll)k * WG + w * 64)),
                                                 16, 0, 0);
        }
        a.cached |= 2;
    }
    if (threadIdx.x == 0) {
        if (direct) cx.st->n_direct += 1;
        else cx.st->n_fft += 1;
        cx.sh->jargs[slot] = a;
        cx.sh->pub[slot] = publish ? 1 : 2;
        if (publish) {
            const int ji = blockIdx.x * JPW + slot;
            Job *jb = cx.pl.jobs + ji;
            const unsigned long long *aw = (const unsigned long long *)&a;
            for (int k = 0; k < (int)(sizeof(JobArgs) / 8); ++k)
                __hip_atomic_exchange((unsigned long long *)&jb->a + k, aw[k], __ATOMIC_RELAXED, AGENT);
            for (int k = 0; k < 3; ++k) __hip_atomic_exchange(&jb->done[k], 0u, __ATOMIC_RELAXED, AGENT);
            const unsigned gen = cx.sh->gen[slot] + 1;
            cx.sh->gen[slot] = gen;
            __hip_atomic_exchange(&jb->ctl, mkctl(gen, 0, 0, a.ntile), __ATOMIC_RELEASE, AGENT);
            flag_slot(cx.pl, ji);
            cx.st->n_published += 1;
        }
    }
    __syncthreads();
    return need;
}

// The cached kernel spectrum of an h-step correlation of 2^lgN points (all
// threads call; filled on a miss, oldest entry replaced).
__device__ __forceinline__ const double2 *spec_get(const Ctx &cx, ll h, int lgN, bool pin)
{
    static_assert(SPC_E <= 64, "one key per lane of wave 0");
    if (threadIdx.x < 64) {
        // lane k compares key k; the highest matching entry wins
        const ll key = (h << 8) | lgN;
        const int l = threadIdx.x;
        const unsigned long long hit = __ballot(l < SPC_E && cx.sh->spk[l < SPC_E ? l : 0] == key);
        if (l == 0) {
            int x = hit ? 63 - __clzll(hit) : -1;
            cx.sh->spf = x < 0;
            if (x < 0) {
                // the oldest entry that no outstanding published job reads
                for (int k = 0; k < SPC_E && x < 0; ++k) {
                    const int y = cx.sh->spn % SPC_E;
                    cx.sh->spn += 1;
                    if (cx.sh->spin[y] == 0) x = y;
                }
                if (x >= 0) cx.sh->spk[x] = key;
            }
            if (pin && x >= 0) cx.sh->spin[x] += 1;
            cx.sh->spx = x;
        }
    }
    __syncthreads();
    const int x = __builtin_amdgcn_readfirstlane(cx.sh->spx);
    if (x < 0) return nullptr;  // every entry is read by an outstanding job
    double2 *e = cx.spc + (ll)x * cx.spc_ent;
    if (__builtin_amdgcn_readfirstlane(cx.sh->spf)) {
        spec_fill(cx.p, h, lgN, e, cx.twl, cx.tw);
        sync_stores();
    }
    return e;
}

// The published job of `slot` no longer reads its spectrum-cache entry (thread 0).
__device__ __forceinline__ void unpin_spec(const Ctx &cx, int slot)
{
    const int x = cx.sh->sppub[slot];
    if (x >= 0) {
        cx.sh->spin[x] -= 1;
        cx.sh->sppub[slot] = -1;
    }
}

// Finish the pending job of `slot`: a private job's tiles are computed here
// in order; for a published one the driver takes the tiles no other
// workgroup has claimed and waits for the rest.
template <int PREC>
__device__ __forceinline__ void conv_wait(const Ctx &cx, int slot)
{
    const int mode = __builtin_amdgcn_readfirstlane(cx.sh->pub[slot]);
    if (mode == 0) return;
    const JobArgs a = uni_args(cx.sh->jargs[slot]);
    const int ji = blockIdx.x * JPW + slot;
    Job *jb = cx.pl.jobs + ji;
    const ll t0 = clk();
    // a private FP64 transform takes its kernel spectrum from the cache
    const bool cached = PREC == 0 && mode == 2 && a.kind != K_DIRECT && a.lgN <= SPC_LG &&
                        __builtin_amdgcn_readfirstlane(a.beta == 0.0 ? 1 : 0);
    // a published one may carry it (the driver's cache entry, pinned)
    const double2 *spec = cached ? spec_get(cx, a.h, a.lgN)
                                 : ((a.kind == K_LDS && (a.cached & 1)) ? (const double2 *)a.scr : nullptr);
    const ll deadline = now_ticks() + cx.tn.timeout_ticks;
    ll work = 0;
    int nph = 0, nt = 0;  // private: next tile
    for (;;) {
        int msg;  // 1 done, 2 tile (phase, index), 3 abort, 0 nothing yet
        if (mode == 2) {
            msg = (nph < a.nph) ? (2 | (nph << 4) | (nt << 8)) : 1;
            if (++nt == a.ntile) {
                nt = 0;
                ++nph;
            }
        } else {
            if (threadIdx.x < 64) {
                int m = 0, ph = 0, t = 0;
                if (threadIdx.x == 0) {
                    const unsigned long long c = rmw_read(&jb->ctl);
                    const unsigned p = ctl_ph(c);
                    if (p == PH_DONE) {
                        fence_acq();
                        m = 1;
                    } else if (p < 3 && ctl_claimed(c) < ctl_total(c) && claim_tile(cx.pl, ji, &ph, &t)) {
                        m = 2 | (ph << 4) | (t << 8);
                    } else if (aborted(cx.pl)) {
                        m = 3;
                    } else if (now_ticks() > deadline) {
                        note_abort(cx.pl, 2, ji, (ll)c, ((ll)a.nph << 32) | (ll)(unsigned)a.ntile,
                                   ((ll)a.kind << 32) | (ll)(unsigned)a.lgN, blockIdx.x, slot);
                        m = 3;
                    } else {
                        __builtin_amdgcn_s_sleep(1);
                    }
                    cx.sh->msg = m;
                }
            }
            __syncthreads();
            msg = __builtin_amdgcn_readfirstlane(cx.sh->msg);
            __syncthreads();
        }
        if ((msg & 15) == 1) break;
        if ((msg & 15) == 3) {
            set_err(cx, DEV_TIMEOUT);
            break;
        }
        if ((msg & 15) == 2) {
            const ll tb = clk();
            run_tile<PREC>(cx.p, a, (msg >> 4) & 15, msg >> 8, cx.lds, cx.tw, cx.twl, cx.twf, spec);
            if (mode == 1) {
                sync_stores();
                if (threadIdx.x == 0) complete_tile(cx.pl, ji, (msg >> 4) & 15, a.ntile, a.nph);
            }
            work += clk() - tb;
        }
    }
    if (threadIdx.x == 0) {
        cx.sh->pub[slot] = 0;
        unpin_spec(cx, slot);
        cx.st->cyc_tiles += work;
        cx.st->cyc_wait += clk() - t0 - work;
    }
    __syncthreads();
}

// After an error: retire every pending job of this workgroup without computing
// it (published ones by claiming and completing their remaining tiles, so
// that no other workgroup still works on the slot when it is reused).
__device__ __forceinline__ void drain(const Ctx &cx)
{
    if (threadIdx.x == 0) {
        const ll deadline = now_ticks() + cx.tn.timeout_ticks;
        for (int slot = 0; slot < JPW; ++slot) {
            if (cx.sh->pub[slot] == 1) {
                const int ji = blockIdx.x * JPW + slot;
                Job *jb = cx.pl.jobs + ji;
                const JobArgs &a = cx.sh->jargs[slot];
                for (;;) {
                    const unsigned long long c = rmw_read(&jb->ctl);
                    const unsigned p = ctl_ph(c);
                    int ph, t;
                    if (p == PH_DONE) break;
                    if (p < 3 && ctl_claimed(c) < ctl_total(c) && claim_tile(cx.pl, ji, &ph, &t)) {
                        complete_tile(cx.pl, ji, ph, a.ntile, a.nph);
                    } else if (aborted(cx.pl)) {
                        break;
                    } else if (now_ticks() > deadline) {
                        note_abort(cx.pl, 3, ji, (ll)c, ((ll)a.nph << 32) | (ll)(unsigned)a.ntile, 0, blockIdx.x, slot);
                        break;
                    } else {
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
            }
            cx.sh->pub[slot] = 0;
            unpin_spec(cx, slot);
        }
    }
    __syncthreads();
}

// Read one double a pool job wrote (after conv_wait's acquire), with an
// atomic read-modify-write like the pool's shared words.
__device__ __forceinline__ double read_result(const double *p)
{
    const unsigned long long v = rmw_read((unsigned long long *)p);
    return __longlong_as_double((long long)v);
}

// Ordering point for one wave's own LDS and global accesses (its earlier
// writes complete before its later reads).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// True if every correlation of a trapezoid of height h with n_red red cells
// (lattices) or boundary-centred width 2h (BSM) is short enough for direct
// stepping, so that one wave can solve it alone.
__device__ __forceinline__ bool wave_sized(const Mp &d, const Tune &tn, ll nred, ll h)
{
    const ll n = (d.model == BSM) ? 2 * h : nred;
    return n <= tn.direct_max_n && n <= DIRECT_MAX_N && h <= 2 * (ll)tn.direct_max_h;
}

#define WGS __HIP_MEMORY_SCOPE_WORKGROUP

// Claim the next unclaimed ticket (one wave; -1 if none).
__device__ __forceinline__ int wq_claim(WQueue *q)
{
    int k = -1;
    if ((threadIdx.x & 63) == 0) {
        const int t = __hip_atomic_load(&q->tail, __ATOMIC_ACQUIRE, WGS);
        int h = __hip_atomic_load(&q->head, __ATOMIC_RELAXED, WGS);
        while (h < t) {
            if (__hip_atomic_compare_exchange_strong(&q->head, &h, h + 1, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED, WGS)) {
                k = h;
                break;
            }
        }
    }
    return __builtin_amdgcn_readfirstlane(k);
}

// Run the part of claimed ticket k and count it done (its global writes complete first).
__device__ __forceinline__ void wq_run(const Mp &d, WQueue *q, int k)
{
    const int e = __builtin_amdgcn_readfirstlane(q->ticket[k % WQT]);
    const int slot = e & 255, part = (e >> 8) & 255, parts = e >> 16;
    WJob j = q->job[slot];
    j.n_in = uni(j.n_in);
    j.h = uni(j.h);
    j.out_off = uni(j.out_off);
    j.n_out = uni(j.n_out);
    direct_part(d, j.src, j.n_in, j.h, j.out_off, j.n_out, j.dst, part, parts);
    wave_sync();
    if ((threadIdx.x & 63) == 0) __hip_atomic_fetch_sub(&q->left[slot], 1, __ATOMIC_RELEASE, WGS);
}

// A helper wave of a small-trapezoid solve: run queued correlations until the
// solving wave has finished (or a deadline passes).
__device__ __forceinline__ void wq_worker(const Mp &d, WQueue *q, ll timeout_ticks)
{
    ll last = now_ticks();
    for (;;) {
        const int k = wq_claim(q);
        if (k >= 0) {
            wq_run(d, q, k);
            last = now_ticks();
            continue;
        }
        int stop = 0;
        if ((threadIdx.x & 63) == 0) {
            stop = __hip_atomic_load(&q->quit, __ATOMIC_ACQUIRE, WGS) &&
                   __hip_atomic_load(&q->head, __ATOMIC_RELAXED, WGS) >= __hip_atomic_load(&q->tail, __ATOMIC_RELAXED, WGS);
            if (now_ticks() - last > timeout_ticks) stop = 1;
        }
        if (__builtin_amdgcn_readfirstlane(stop)) break;
    }
}

// Push the job of stack slot `slot` (the solving wave); returns its first
// ticket.  A lattice job gets one ticket per output segment while the ring
// has room for them (else one ticket that steps every segment); a BSM job
// keeps one ticket, since its segments overlap by a halo on both sides and
// its waves are kept busy by the many short correlations of the cone.
__device__ __forceinline__ int wq_push(const Mp &d, WQueue *q, int slot, const WJob &j, int *tail)
{
    const int k = *tail;
    int parts = (d.model == BSM) ? 1 : direct_nseg(d, j.n_in, j.h, j.n_out);
    if (parts > 1) {
        int hd = 0;
        if ((threadIdx.x & 63) == 0) hd = __hip_atomic_load(&q->head, __ATOMIC_RELAXED, WGS);
        hd = __builtin_amdgcn_readfirstlane(hd);
        if (k - hd + parts > WQT) parts = 1;
    }
    if ((threadIdx.x & 63) == 0) {
        q->job[slot] = j;
        q->left[slot] = parts;
        for (int p = 0; p < parts; ++p) q->ticket[(k + p) % WQT] = slot | (p << 8) | (parts << 16);
    }
    wave_sync();  // the entry and this wave's row writes precede the publication
    if ((threadIdx.x & 63) == 0) __hip_atomic_store(&q->tail, k + parts, __ATOMIC_RELEASE, WGS);
    *tail = k + parts;
    return k;
}

// Wait for the job of slot `slot` (the solving wave), running unclaimed
// tickets meanwhile.
__device__ __forceinline__ bool wq_wait(const Mp &d, WQueue *q, int slot, ll timeout_ticks, Stats *st)
{
    const ll t0 = now_ticks();
    for (;;) {
        int fin = 0;
        if ((threadIdx.x & 63) == 0) fin = __hip_atomic_load(&q->left[slot], __ATOMIC_ACQUIRE, WGS) == 0;
        if (__builtin_amdgcn_readfirstlane(fin)) return true;
        const int c = wq_claim(q);
        if (c >= 0) {
            const ll tb = clk();
            wq_run(d, q, c);
            if ((threadIdx.x & 63) == 0) st->cyc_tiles += clk() - tb;
            continue;
        }
        if (now_ticks() - t0 > timeout_ticks) return false;
    }
}

// A frame's scalar fields as wave-uniform values.
__device__ __forceinline__ Frame uni_frame(Frame fr)
{
    fr.r0 = uni(fr.r0);
    fr.c0 = uni(fr.c0);
    fr.h = uni(fr.h);
    fr.b = uni(fr.b);
    fr.aoff = uni(fr.aoff);
    fr.soff = uni(fr.soff);
    fr.stage = __builtin_amdgcn_readfirstlane(fr.stage);
    return fr;
}

// Wave-local solve of a small trapezoid (see wave_sized): wave 0 alone walks
// the frame stages of solve_trapezoid -- first correlation, first
// sub-trapezoid, second correlation, second sub-trapezoid -- stepping each
// correlation directly and walking the band at the leaves, with its stack in
// LDS at wstk (cap frames) and no workgroup barrier.  Returns the boundary of
// the last row; on a failed check lane 0 records the error in *cx.err_sh.
__device__ __forceinline__ ll wave_solve(const Ctx &cx, Frame root, Frame *wstk, int cap, WQueue *q)
{
    const Mp d = cx.p;
    const int l = threadIdx.x & 63;
    // a lattice frame steps kstep rows at a time (a Bermudan binomial call: from
    // one exercise row to the next) and its cone widens by span columns per step
    const ll kstep = (d.model == BINOMIAL && d.ex_every > 1) ? d.ex_every : 1;
    const ll span = (d.model == BINOMIAL) ? kstep : 2;
    const ll timeout = cx.tn.timeout_ticks;
    const ll bw = band_width(d);
    if (cap > WQ) cap = WQ;  // one outstanding correlation per frame fits the queue
    // The frame being worked on (depth sp) lives in registers; the stack
    // holds its ancestors, each stored when its child was entered.
    int sp = 0, tail = 0;
    ll rv = 0;
    int e = DEV_OK;
    // work counters, kept in registers of lane 0 and added to the LDS ones on return
    ll n_conv = 0, c_in = 0, c_out = 0, c_pts = 0, b_rows = 0, b_cyc = 0;
    // a leaf: the band walk over the trapezoid's rows (ranges already checked)
    auto walk = [&](const Frame &f) -> ll {
        const ll tb = clk();
        ll r;
        if (d.model == BINOMIAL) r = band_bin(d, f.r0, f.c0, kstep * f.h, f.b, f.src, f.dst, cx.bnd, nullptr);
        else if (d.model == TRINOMIAL) r = band_tri(d, f.r0, f.c0, f.h, f.b, f.src, f.dst, cx.bnd, nullptr);
        else r = band_bsm(d, f.r0, f.c0, f.h, f.c0 + 2 * f.h, f.src, f.dst, cx.bnd, nullptr);
        if (l == 0) {
            b_rows += kstep * f.h;
            b_cyc += clk() - tb;
        }
        return uni(r);
    };
    // leaf test and its range checks (lattice: red cells [c0, b]; BSM: centred on c0)
    auto is_leaf = [&](const Frame &f) -> bool {
        return (d.model != BSM) ? (f.b - f.c0 + 1 <= bw) : (f.h <= (bw - 2) / 2);
    };
    auto leaf_ok = [&](const Frame &f) -> bool {
        return (d.model != BSM) ? (in_ws(cx, f.src, f.c0, f.b) && in_ws(cx, f.dst, f.c0, f.c0 + bw - 1))
                                : (in_ws(cx, f.src, f.c0 + 1, f.c0 + 2 * f.h) && in_ws(cx, f.dst, f.c0 - f.h, f.c0 + f.h));
    };
    Frame fr = uni_frame(root);
    for (;;) {
        // the frame's pending correlation (job index + 1 in soff) must be done
        // before its next stage reads its output
        if (fr.soff > 0) {
            if (!wq_wait(d, q, sp, timeout, cx.st)) {
                e = DEV_TIMEOUT;
                break;
            }
            fr.soff = 0;
        }
        bool pop = false, leaf = false;
        Frame child;
        const double *csrc = nullptr;
        double *cdst = nullptr;
        ll cn = 0, ch = 0, coff = 0, cout = 0;
        if (d.model != BSM) {
            const ll i0 = fr.r0, c0 = fr.c0, h = fr.h, b = fr.b;
            const ll h1 = h / 2, h2 = h - h1;
            const ll nred = b - c0 + 1;
            if (fr.stage == 0) {
                if (nred <= bw) {  // only a root can be a leaf: children that are leaves are walked inline
                    if (!leaf_ok(fr)) e = DEV_RANGE;
                    else leaf = true;
                    pop = true;
                } else {
                    double *mid = cx.arena + fr.aoff - c0;
                    if (fr.aoff + nred > cx.arena_len) e = DEV_ARENA;
                    else if (!in_ws(cx, fr.src, c0, b)) e = DEV_RANGE;
                    else {
                        csrc = fr.src + c0;
                        cn = nred;
                        ch = kstep * h1;
                        coff = (d.model == BINOMIAL) ? 0 : h1;
                        cout = nred - span * h1;
                        cdst = mid + c0;
                        fr.mid = mid;
                        fr.stage = 1;
                        child = Frame{i0, b - span * h1 + 1, h1, b, fr.aoff + nred, 0, fr.src, mid, nullptr, 0, 0};
                    }
                }
            } else if (fr.stage == 1) {
                const ll br = rv;
                const ll n2 = br - c0 + 1;
                if (!in_ws(cx, fr.mid, c0, br) || !in_ws(cx, fr.dst, c0, br)) e = DEV_RANGE;
                else {
                    csrc = fr.mid + c0;
                    cn = n2;
                    ch = kstep * h2;
                    coff = (d.model == BINOMIAL) ? 0 : h2;
                    cout = n2 - span * h2;
                    cdst = fr.dst + c0;
                    fr.stage = 2;
                    child = Frame{i0 - kstep * h1, br - span * h2 + 1, h2, br, fr.aoff + nred, 0, fr.mid, fr.dst,
                                  nullptr, 0, 0};
                }
            } else {
                pop = true;  // rv: the second sub-trapezoid's boundary
            }
        } else {
            const ll n = fr.r0, f = fr.c0, h = fr.h;
            const ll h1 = h / 2, h2 = h - h1;
            if (fr.stage == 0) {
                if (h <= (bw - 2) / 2) {  // only a root can be a leaf
                    if (!leaf_ok(fr)) e = DEV_RANGE;
                    else leaf = true;
                    pop = true;
                } else {
                    const ll base = f - h1 + 1;
                    double *mid = cx.arena + fr.aoff - base;
                    if (fr.aoff + 2 * h > cx.arena_len) e = DEV_ARENA;
                    else if (!in_ws(cx, fr.src, f + 1, f + 2 * h)) e = DEV_RANGE;
                    else {
                        csrc = fr.src + f + 1;
                        cn = 2 * h;
                        ch = h1;
                        coff = h1;
                        cout = 2 * h - 2 * h1;
                        cdst = mid + f + 1 + h1;
                        fr.mid = mid;
                        fr.stage = 1;
                        child = Frame{n, f, h1, 0, fr.aoff + 2 * h, 0, fr.src, mid, nullptr, 0, 0};
                    }
                }
            } else if (fr.stage == 1) {
                const ll fp = rv;
                const ll nin = f + h + h2 - fp;
                if (fp < f - h1 || fp > f) e = DEV_RANGE;
                else if (!in_ws(cx, fr.mid, fp + 1, f + h + h2) || !in_ws(cx, fr.dst, fp + 1 + h2, f + h)) e = DEV_RANGE;
                else {
                    csrc = fr.mid + fp + 1;
                    cn = nin;
                    ch = h2;
                    coff = h2;
                    cout = nin - 2 * h2;
                    cdst = fr.dst + fp + 1 + h2;
                    fr.stage = 2;
                    child = Frame{n + h1, fp, h2, 0, fr.aoff + 2 * h, 0, fr.mid, fr.dst, nullptr, 0, 0};
                }
            } else {
                pop = true;
            }
        }
        if (e != DEV_OK) break;
        if (!pop && cout > 0) {
            // the stage's correlation goes to the other waves while this one
            // solves the sub-trapezoid that does not depend on it
            WJob j;
            j.src = csrc;
            j.dst = cdst;
            j.n_in = cn;
            j.h = ch;
            j.out_off = coff;
            j.n_out = cout;
            fr.soff = wq_push(d, q, sp, j, &tail) + 1;
            if (l == 0) {
                const int lg = ceil_log2(cn);
                n_conv += 1;
                c_in += cn;
                c_out += cout;
                c_pts += ll(1) << (lg < 1 ? 1 : lg);
            }
        }
        // A child that is a leaf is walked right here, after the push above
        // (so the correlation overlaps it), and this frame stays current for
        // its next stage; a root that is a leaf is walked the same way.
        const bool inl = !pop && is_leaf(child);
        if (inl && !leaf_ok(child)) {
            e = DEV_RANGE;
            break;
        }
        if (leaf || inl) rv = walk(inl ? child : fr);
        if (pop) {
            if (sp == 0) break;
            --sp;
            fr = uni_frame(wstk[sp]);
        } else if (inl) {
        } else if (sp + 1 >= cap) {
            e = DEV_STACK;
            break;
        } else {
            if (l == 0) wstk[sp] = fr;  // read back by this wave only, after the child's subtree
            ++sp;
            fr = child;
        }
    }
    if (e != DEV_OK && e != DEV_TIMEOUT) {
        // finish the outstanding jobs of this frame and of its ancestors
        bool ok = fr.soff <= 0 || wq_wait(d, q, sp, timeout, cx.st);
        for (int k = sp - 1; ok && k >= 0; --k) {
            const ll so = uni(wstk[k].soff);
            if (so > 0) ok = wq_wait(d, q, k, timeout, cx.st);
        }
    }
    if (l == 0) {
        Stats *st = cx.st;
        st->convs += n_conv;
        st->n_direct += n_conv;
        st->conv_in += c_in;
        st->conv_out += c_out;
        st->fft_points += c_pts;
        st->band_rows += b_rows;
        st->cyc_band += b_cyc;
        if (e != DEV_OK && *cx.err_sh == 0) *cx.err_sh = e;
    }
    return rv;
}

// Solve one trapezoid (model-dependent geometry, see the frame stages below)
// and return the boundary of its last row.  All lanes call it; control flow is
// uniform.  A frame at depth s keeps its correlations in job slot s + 1: the
// first one is computed while the first sub-trapezoid is solved, the second
// while the second is, and the frame ends only after both are done.  Each
// iteration first finishes the frame's pending correlation (stages 1 and 2),
// then takes the frame one stage further, which may submit one correlation.
template <int PREC>
__device__ __forceinline__ ll solve_trapezoid(const Ctx &cx, Frame root, Frame *stk, int *sp_sh, ll *ret_sh,
                                              ll *leaf_sh, ll *red_sh)
{
    const Mp d = cx.p;
    const int tid = threadIdx.x;
    // lattice frames step kstep rows at a time (a Bermudan binomial call: from
    // one exercise row to the next); the cone widens by span columns per step
    const ll kstep = (d.model == BINOMIAL && d.ex_every > 1) ? d.ex_every : 1;
    const ll span = (d.model == BINOMIAL) ? kstep : 2;
    if (tid == 0) {
        stk[0] = root;
        *sp_sh = 0;
    }
    __syncthreads();
    int iter = 0;
    for (;;) {
        const int s = *sp_sh;
        if (s < 0 || *cx.err_sh) break;
        if (tid == 0 && cx.tn.late_pub_lg > 0 && !cx.sh->late && (++iter & 15) == 0 &&
            (int)(rmw_read((unsigned long long *)&cx.pl.hdr->status) & 0xffffffffull) >= cx.tn.late_after)
            cx.sh->late = 1;
        Frame fr = stk[s];
        fr.r0 = uni(fr.r0);
        fr.c0 = uni(fr.c0);
        fr.h = uni(fr.h);
        fr.b = uni(fr.b);
        fr.aoff = uni(fr.aoff);
        fr.soff = uni(fr.soff);
        fr.stage = __builtin_amdgcn_readfirstlane(fr.stage);
        const int slot = s + 1;
        const ll rv = uni(*ret_sh);
        __syncthreads();
        if (fr.stage > 0) conv_wait<PREC>(cx, slot);
        bool pop = false, leaf = false;
        ll result = 0;
        Frame child;
        int e = DEV_OK;
        // the correlation this step submits, if any
        const double *csrc = nullptr;
        double *cdst = nullptr;
        ll cn = 0, ch = 0, coff = 0, cout = 0;
        if (d.model != BSM) {
            // Lattice trapezoid (i0 = r0): red cells [c0, b] of row i0 in src;
            // produces the red cells of row i0 - h in dst.
            const ll i0 = fr.r0, c0 = fr.c0, h = fr.h, b = fr.b;
            const ll h1 = h / 2, h2 = h - h1;
            const ll nred = b - c0 + 1;
            if (fr.stage == 0) {
                if (nred <= band_width(d) || (kstep <= BAND && wave_sized(d, cx.tn, nred, kstep * h))) {
                    leaf = true;  // wave 0 solves it alone (band, or direct steps and bands)
                    pop = true;
                } else if (kstep > 1 && h == 1) {
                    // One exercise interval of a Bermudan call over more red
                    // cells than a band holds (kstep > BAND): the cells right
                    // of b are exercise cells of row i0, so the red cells
                    // extended by their exercise values are correlated over
                    // kstep rows in one piece, then the max is taken on the
                    // exercise row below.
                    const ll wext = (b + kstep < i0) ? b + kstep : i0;  // last column read on row i0
                    const ll n_in = wext - c0 + 1, n_out = n_in - kstep, i1 = i0 - kstep;
                    double *ext = cx.arena + fr.aoff;
                    if (n_out < 1) {
                        // row i1 ends left of c0: its cells are all continuation
                        // cells of the parent's left part, and its boundary is its end
                        if (cx.bnd)
                            for (ll i = i1 + tid; i < i0; i += WG) cx.bnd[i] = i;
                        result = i1;
                        pop = true;
                    } else if (fr.aoff + n_in > cx.arena_len || slot >= JPW) e = DEV_ARENA;
                    else if (!in_ws(cx, fr.src, c0, b) || !in_ws(cx, fr.dst, c0, c0 + n_out - 1))
                        e = DEV_RANGE;
                    else {
                        for (ll k = tid; k < n_in; k += WG)
                            ext[k] = (c0 + k <= b) ? fr.src[c0 + k] : ex_bin(d, i0, c0 + k);
                        __syncthreads();
                        // tilted about the strike column (the exercise values grow like u^{2j})
                        double tc = 0.5 * ((double)i0 + log(d.K / d.S) / d.a) - (double)c0;
                        tc = tc < 0.0 ? 0.0 : (tc > (double)(n_in - 1) ? (double)(n_in - 1) : tc);
                        conv_submit<PREC>(cx, slot, fr.soff, ext, n_in, kstep, 0, n_out, fr.dst + c0, 2.0 * d.a, tc);
                        conv_wait<PREC>(cx, slot);
                        ll last = c0 - 1;
                        for (ll k = tid; k < n_out; k += WG) {
                            const ll j = c0 + k;
                            const double c = fr.dst[j], ee = ex_bin(d, i1, j);
                            const bool red = red_of(c, ee);
                            fr.dst[j] = red ? c : ee;
                            if (red && j > last) last = j;
                        }
                        last = block_max(last, red_sh);
                        if (cx.bnd) {
                            for (ll i = i1 + 1 + tid; i < i0; i += WG) cx.bnd[i] = i;  // rows without exercise
                            if (tid == 0) cx.bnd[i1] = last;
                        }
                        if (tid == 0) cx.st->band_rows += kstep;
                        result = last;
                        pop = true;
                    }
                } else {
                    // (1) row r = i0 - h1, columns [c0, b - span h1], by correlation from row i0.
                    double *mid = cx.arena + fr.aoff - c0;
                    if (fr.aoff + nred > cx.arena_len || slot >= JPW) e = DEV_ARENA;
                    else if (!in_ws(cx, fr.src, c0, b)) e = DEV_RANGE;
                    else {
                        csrc = fr.src + c0;
                        cn = nred;
                        ch = kstep * h1;
                        coff = (d.model == BINOMIAL) ? 0 : h1;
                        cout = nred - span * h1;
                        cdst = mid + c0;
                        fr.mid = mid;
                        fr.stage = 1;
                        // (2) sub-trapezoid on the last span*h1 red cells of row i0
                        child = Frame{i0, b - span * h1 + 1, h1, b, fr.aoff + nred, 0, fr.src, mid, nullptr, 0, 0};
                    }
                }
            } else if (fr.stage == 1) {
                // (3) row i0 - h, columns [c0, br - span h2], by correlation from row r.
                const ll br = rv;
                const ll n2 = br - c0 + 1;
                if (!in_ws(cx, fr.mid, c0, br) || !in_ws(cx, fr.dst, c0, br)) e = DEV_RANGE;
                else {
                    csrc = fr.mid + c0;
                    cn = n2;
                    ch = kstep * h2;
                    coff = (d.model == BINOMIAL) ? 0 : h2;
                    cout = n2 - span * h2;
                    cdst = fr.dst + c0;
                    fr.stage = 2;
                    // (4) sub-trapezoid on the last span*h2 red cells of row r
                    child = Frame{i0 - kstep * h1, br - span * h2 + 1, h2, br, fr.aoff + nred, 0, fr.mid, fr.dst,
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
                if (h <= (BAND2 - 2) / 2 || wave_sized(d, cx.tn, 2 * h, h)) {
                    leaf = true;  // wave 0 solves it alone
                    pop = true;
                } else {
                    // middle step n+h1 on [f-h1+1, f+h+h2] (2h cells)
                    const ll base = f - h1 + 1;
                    double *mid = cx.arena + fr.aoff - base;
                    if (fr.aoff + 2 * h > cx.arena_len || slot >= JPW) e = DEV_ARENA;
                    else if (!in_ws(cx, fr.src, f + 1, f + 2 * h)) e = DEV_RANGE;
                    else {
                        // conv 1: red cells [f+1, f+2h] -> [f+1+h1, f+2h-h1] of step n+h1
                        csrc = fr.src + f + 1;
                        cn = 2 * h;
                        ch = h1;
                        coff = h1;
                        cout = 2 * h - 2 * h1;
                        cdst = mid + f + 1 + h1;
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
                    csrc = fr.mid + fp + 1;
                    cn = nin;
                    ch = h2;
                    coff = h2;
                    cout = nin - 2 * h2;
                    cdst = fr.dst + fp + 1 + h2;
                    fr.stage = 2;
                    child = Frame{n + h1, fp, h2, 0, fr.aoff + 2 * h, 0, fr.mid, fr.dst, nullptr, 0, 0};
                }
            } else {
                result = rv;
                pop = true;
            }
        }
        if (leaf) {
            WQueue *q = &cx.sh->wq;
            if (tid == 0) {
                q->head = 0;
                q->tail = 0;
                q->quit = 0;
                for (int k = 0; k < WQ; ++k) q->left[k] = 0;
            }
            __syncthreads();
            if (tid < 64) {
                // wave 0 solves; waves 1..3 step the correlations it queues
                Frame w = fr;
                w.stage = 0;
                w.soff = 0;
                const ll r = wave_solve(cx, w, stk + s + 1, MAXD - s - 1, q);
                if (tid == 0) {
                    *leaf_sh = r;
                    __hip_atomic_store(&q->quit, 1, __ATOMIC_RELEASE, WGS);
                }
            } else {
                wq_worker(d, q, cx.tn.timeout_ticks);
            }
            __syncthreads();
            result = *leaf_sh;
        }
        if (e == DEV_OK && !pop && cout > 0) {
            // the child is solved at wave level (no FFT tile runs before this
            // correlation is waited for): its input may be staged in LDS
            const bool child_wave = (d.model != BSM)
                                        ? (child.b - child.c0 + 1 <= band_width(d) ||
                                           (kstep <= BAND && wave_sized(d, cx.tn, child.b - child.c0 + 1, kstep * child.h)))
                                        : (child.h <= (BAND2 - 2) / 2 || wave_sized(d, cx.tn, 2 * child.h, child.h));
            child.soff = fr.soff + conv_submit<PREC>(cx, slot, fr.soff, csrc, cn, ch, coff, cout, cdst, 0.0, 0.0,
                                                     child_wave);
        }
        else if (!pop)
            child.soff = fr.soff;
        if (tid == 0) {
            if (e != DEV_OK) {
                if (*cx.err_sh == 0) *cx.err_sh = e;
            } else if (pop) {
                *ret_sh = result;
                *sp_sh = s - 1;
            } else if (s + 1 >= MAXD) {
                *cx.err_sh = DEV_STACK;
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
template <int PREC>
__device__ __forceinline__ double drive_lattice(const Ctx &cx, double *rowA, double *rowB, Frame *stk, int *sp_sh,
                                                ll *ret_sh, ll *leaf_sh, ll *red_sh, double *val_sh)
{
    const Mp d = cx.p;
    const ll T = d.T;
    const int tid = threadIdx.x;
    const bool bin = d.model == BINOMIAL;
    const ll wT = bin ? T : 2 * T;  // last column of row T
    const int ev = d.ex_every;      // 1 American, 0 European, >= 2 Bermudan (binomial)
    const bool berm = ev > 1;
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
            // European or Bermudan: row T-1 has no exercise
            const bool red = ev != 1 || red_of(c, e);
            rowA[j] = red ? c : e;
            if (red) lastT1 = j;
        }
    }
    if (tid == 0) cx.st->direct_cells += wT + 1 - (bin ? 1 : 2);
    lastT = block_max(lastT, red_sh);
    lastT1 = block_max(lastT1, red_sh);
    if (cx.bnd && tid == 0) {
        cx.bnd[T] = lastT;
        cx.bnd[T - 1] = ev == 0 ? -1 : lastT1;
    }
    if (tid == 0) cx.st->cyc_rows += clk() - tr0;
    ll i0 = T - 1, b = lastT1;
    double *src = rowA, *dst = rowB;
    // strike column of row i (binomial), the centre of a tilted correlation
    auto strike_col = [&](ll i, ll last) {
        double tc = 0.5 * ((double)i + log(d.K / d.S) / d.a);
        return tc < 0.0 ? 0.0 : (tc > (double)last ? (double)last : tc);
    };
    if (T > 1 && (d.no_green || ev == 0 || (berm && ev > T) || (ev == 1 && b == wT - (bin ? 1 : 2)))) {
        // No exercise cell below the expiry row: with Y = 0 Lemma 2.3 leaves
        // none (the classification of far in-the-money cells of row T-1 is
        // then rounding noise), and an entirely red row T-1 keeps every row
        // below red (Corollary 2.6: the boundary drops at most one cell per
        // row while the row shrinks by one or two).  The root is then one
        // linear functional of row T-1, whose values grow like S u^{col}, so
        // the correlation is tilted about the at-the-money column tc.  A
        // European option (exercise at expiry only) takes the same single
        // correlation: row T-1 was computed without exercise; so does a
        // Bermudan option with no exercise row below the expiry row.
        b = wT - (bin ? 1 : 2);
        if (cx.bnd && tid == 0) cx.bnd[T - 1] = ev == 0 ? -1 : b;
        const double beta = bin ? 2.0 * d.a : d.a;
        double tc = bin ? 0.5 * ((double)(T - 1) + log(d.K / d.S) / d.a)
                        : (double)(T - 1) + log(d.K / d.S) / d.a;
        if (tc < 0.0) tc = 0.0;
        if (tc > (double)b) tc = (double)b;
        if (cx.bnd)
            for (ll i = tid; i < T - 1; i += WG) cx.bnd[i] = ev == 0 ? -1 : (bin ? i : 2 * i);
        const ll hh = T - 1;
        conv_submit<PREC>(cx, SLOT_TOP, 0, src, b + 1, hh, bin ? 0 : hh, 1, dst, beta, tc);
        conv_wait<PREC>(cx, SLOT_TOP);
        if (tid == 0) *val_sh = read_result(dst);
        __syncthreads();
        return *val_sh;
    }
    // Bermudan binomial call: the rows between exercise rows carry no
    // exercise, so the recursion steps from one exercise row to the next (ev
    // rows, whose kernel is the ev-step binomial one; the cone widens by ev
    // columns per step).  The first exercise row below expiry, i1 = T - ev,
    // is computed directly: row T-1 (linear) correlated over ev - 1 rows,
    // tilted like the Y = 0 case (the row is linear up to its top), then the
    // max with the exercise values.
    const ll r0 = berm ? T % ev : 0;  // lowest exercise row
    // The exercise row i0 (red cells [0, b] in src) stepped to row tgt = i0 - s
    // through the whole row: the cells right of b are exercise cells, whose
    // values enter; then, if tgt exercises, the max and the boundary.
    auto full_step = [&](ll s, double *from, double *to) -> ll {
        for (ll j = b + 1 + tid; j <= i0; j += WG) from[j] = ex_bin(d, i0, j);
        __syncthreads();
        const ll tgt = i0 - s;
        conv_submit<PREC>(cx, SLOT_TOP, 0, from, i0 + 1, s, 0, tgt + 1, to, 2.0 * d.a, strike_col(i0, i0));
        conv_wait<PREC>(cx, SLOT_TOP);
        ll last = -1;
        const bool exr = (T - tgt) % ev == 0;
        for (ll j = tid; j <= tgt; j += WG) {
            const double c = to[j], e = ex_bin(d, tgt, j);
            const bool red = !exr || red_of(c, e);
            to[j] = red ? c : e;
            if (red) last = j;
        }
        last = block_max(last, red_sh);
        if (cx.bnd) {
            for (ll i = tgt + 1 + tid; i < i0; i += WG) cx.bnd[i] = i;  // rows without exercise
            if (tid == 0) cx.bnd[tgt] = exr ? last : tgt;
        }
        if (tid == 0) cx.st->direct_cells += tgt + 1;
        __syncthreads();
        return last;
    };
    if (berm) {
        b = full_step(ev - 1, src, dst);  // i0 = T - 1: rows T-1 .. T-ev+1 have no exercise
        i0 = T - ev;
        double *t = src;
        src = dst;
        dst = t;
        if (*cx.err_sh) return NAN;
    }
    while (i0 > 0) {
        if (b < 0) {
            // no red cell: every exercise row below is green (Lemma 2.4).  A
            // Bermudan option's rows without exercise continue linearly from
            // exercise values, down to the root from the lowest exercise row
            // r0: S u^{2j-i} rho_S^n - K rho_K^n at n = r0 rows below it.
            if (cx.bnd)
                for (ll i = tid; i < i0; i += WG) cx.bnd[i] = (berm && (T - i) % ev != 0) ? i : -1;
            __syncthreads();
            if (!berm || r0 == 0) return d.S - d.K;
            const double u = exp(d.a);
            return d.S * exp((double)r0 * log(d.w1 * u + d.w0 / u)) - d.K * exp((double)r0 * log(d.w0 + d.w1));
        }
        const ll nred = b + 1;
        if (nred <= band_width(d)) {  // the band walks the leftover triangle to the root
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
        ll h, rows;
        if (berm) {
            // trapezoid height in exercise intervals, down to the lowest exercise row
            h = nred / ev;
            if (h > (i0 - r0) / ev) h = (i0 - r0) / ev;
            if (h == 0) {
                // the red cells are fewer than one interval, or the lowest
                // exercise row is reached: step through the whole row
                const ll s = (i0 == r0) ? i0 : ev;
                b = full_step(s, src, dst);
                if (*cx.err_sh) return NAN;
                i0 -= s;
                double *t = src;
                src = dst;
                dst = t;
                if (i0 == 0 && (T % ev) != 0) {  // the root is on a row without exercise
                    if (tid == 0) *val_sh = read_result(src);
                    __syncthreads();
                    return *val_sh;
                }
                continue;
            }
            rows = ev * h;
        } else {
            h = bin ? nred : nred / 2;
            if (h > i0) h = i0;
            rows = h;
        }
        Frame root{i0, 0, h, b, 0, 0, src, dst, nullptr, 0, 0};
        if (tid == 0) cx.st->trapezoids += 1;
        b = solve_trapezoid<PREC>(cx, root, stk, sp_sh, ret_sh, leaf_sh, red_sh);
        if (*cx.err_sh) return NAN;
        i0 -= rows;
        double *t = src;
        src = dst;
        dst = t;
    }
    const double p = (b >= 0) ? read_result(src) : d.S - d.K;
    __syncthreads();
    return p;
}

template <int PREC>
__device__ __forceinline__ double drive_bsm(const Ctx &cx, double *rowA, double *rowB, Frame *stk, int *sp_sh,
                                            ll *ret_sh, ll *leaf_sh, ll *red_sh, double *val_sh)
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
            const bool green = d.ex_every != 0 && g > cont;  // European: exercise at expiry only
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
            const double v = (f >= 0) ? ex_bsm(d, 0) : read_result(src);
            __syncthreads();
            return d.K * v;
        }
        if (f < L) {  // no exercise cell left in the cone: the rest is linear
            if (cx.bnd)
                for (ll m = n + 1 + tid; m <= T; m += WG) cx.bnd[m] = NONE;
            const ll hh = T - n;
            conv_submit<PREC>(cx, SLOT_TOP, 0, src + L, R - L + 1, hh, hh, 1, dst);
            conv_wait<PREC>(cx, SLOT_TOP);
            if (tid == 0) *val_sh = read_result(dst);
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
        if (w <= BAND2 - 2) {  // the band walks the leftover cone to the apex
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
        // the rest of step n+h, red cells [f+1+h, R-h] from [f+1, R] of step n,
        // is computed while the trapezoid is solved
        const ll need = conv_submit<PREC>(cx, SLOT_TOP, 0, src + f + 1, w, h, h, w - 2 * h, dst + f + 1 + h);
        Frame root{n, f, h, 0, 0, need, src, dst, nullptr, 0, 0};
        if (tid == 0) cx.st->trapezoids += 1;
        const ll fn = solve_trapezoid<PREC>(cx, root, stk, sp_sh, ret_sh, leaf_sh, red_sh);
        conv_wait<PREC>(cx, SLOT_TOP);
        if (*cx.err_sh) return NAN;
        n += h;
        R -= h;
        L += h;
        f = fn;
        double *t = src;
        src = dst;
        dst = t;
    }
}

// Drive one option (descriptor index o) to its price, with the whole workgroup.
template <int PREC>
__device__ __forceinline__ void drive_option(const Desc &d, ll o, char *ws, const double2 *__restrict__ tw,
                                             double *price, ll *bnd, ll bnd_stride, int32_t *err, Stats *stats,
                                             const Pool &pl, const Tune &tn, double2 *lds, const double2 *twl,
                                             const float4 *twf, Frame *stk, int *sp_sh, int *err_sh, ll *ret_sh, ll *leaf_sh,
                                             ll *red_sh, double *val_sh, Stats *st_sh, Shared *sh)
{
    const int tid = threadIdx.x;
    char *base = ws + d.ws_off;
    if (d.prec != PREC) {  // launched with the other precision's kernel
        if (tid == 0) {
            price[d.out_index] = NAN;
            if (err) err[d.out_index] = DEV_RANGE;
            stats[d.out_index] = Stats{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
            __hip_atomic_fetch_add((unsigned long long *)&pl.hdr->status, 1ull, __ATOMIC_RELEASE, AGENT);
        }
        return;
    }
    double *rowA = (double *)base;
    double *rowB = rowA + d.row_len;
    double *arena = rowB + d.row_len;
    double2 *scr = (double2 *)(arena + d.arena_len);
    Ctx cx;
    cx.p = make_mp(d);
    cx.desc = (int)o;
    cx.lo = rowA;
    cx.hi = (double *)(scr + d.scr_len);
    cx.arena = arena;
    cx.arena_len = d.arena_len;
    cx.scr = scr;
    cx.scr_len = d.scr_len;
    cx.spc = scr + d.scr_len;
    cx.spc_ent = spc_entry(d.nfft);
    cx.lds = lds;
    cx.tw = tw;
    cx.twl = twl;
    cx.twf = twf;
    cx.prec = d.prec;
    cx.bnd = bnd ? bnd + d.out_index * bnd_stride : nullptr;
    cx.st = st_sh;
    cx.pl = pl;
    cx.tn = tn;
    cx.sh = sh;
    cx.err_sh = err_sh;
    if (tid == 0) {
        for (int k = 0; k < SPC_E; ++k) {
            sh->spk[k] = -1;
            sh->spin[k] = 0;
        }
        for (int k = 0; k < JPW; ++k) sh->sppub[k] = -1;
        sh->spn = 0;
        sh->late = 0;
        *err_sh = 0;
        *ret_sh = 0;
        *st_sh = Stats{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    }
    __builtin_amdgcn_s_waitcnt(0);  // no staged input load of a previous option is still in flight
    __syncthreads();
    const ll ttot = clk();
    double p;
    if (d.model == BSM) p = drive_bsm<PREC>(cx, rowA, rowB, stk, sp_sh, ret_sh, leaf_sh, red_sh, val_sh);
    else p = drive_lattice<PREC>(cx, rowA, rowB, stk, sp_sh, ret_sh, leaf_sh, red_sh, val_sh);
    __syncthreads();
    if (*err_sh) drain(cx);
    if (tid == 0) {
        // a refused job or an expired wait anywhere in the launch: nothing
        // finished after it is trusted
        if (!*err_sh && aborted(pl)) *err_sh = DEV_ABORT;
        price[d.out_index] = *err_sh ? NAN : p;
        if (err) err[d.out_index] = *err_sh;
        st_sh->cyc_total = clk() - ttot;
        stats[d.out_index] = *st_sh;
        __hip_atomic_fetch_add((unsigned long long *)&pl.hdr->status, 1ull, __ATOMIC_RELEASE, AGENT);
    }
}

// Persistent solve kernel: options first (one driver workgroup each, claimed
// in descriptor order), then helping with the published jobs of the drivers
// still running.
template <int PREC>
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(1, 1)))
solve_kernel(const Desc *__restrict__ descs, ll n, char *ws, const double2 *__restrict__ tw, double *price, ll *bnd,
             ll bnd_stride, int32_t *err, Stats *stats, Pool pl, Tune tn)
{
    // FFT tiles (FP64: NLDS64 values at padded indices px; mixed: NLDS split-FP32 values)
    __shared__ double2 lds[PREC ? NLDS : NLDS64 + NLDS64 / 8];
    __shared__ double2 twl[NLDS + 1 + (NLDS + 1) / 8 + 1];  // e^{-2 pi i t / 4096} at px(t), t <= 2048
    __shared__ float4 twf[PREC ? NLDS / 2 : 1];  // split twiddles (mixed precision only)
    __shared__ Frame stk[MAXD];
    __shared__ int sp_sh, err_sh;
    __shared__ ll ret_sh, leaf_sh, red_sh[WG / 64];
    __shared__ double val_sh;
    __shared__ Stats st_sh;
    __shared__ Shared sh;

    const int tid = threadIdx.x;
    for (int t = tid; t <= NLDS; t += WG) twl[px(t)] = tw[(ll)t << (LG_TW - LG_NLDS - 1)];
    if (PREC) {
        for (int t = tid; t < NLDS / 2; t += WG) {
            const double2 w = tw[(ll)t << (LG_TW - LG_NLDS)];  // e^{-2 pi i t / 2048}
            const CF c = cf_from(w.x, w.y);
            twf[t] = make_float4(c.rh, c.rl, c.ih, c.il);
        }
    }
    for (int t = tid; t < JPW; t += WG) {
        sh.pub[t] = 0;
        sh.gen[t] = 0;
    }
    __syncthreads();
    for (;;) {
        if (tid == 0) sh.opt = (int)__hip_atomic_fetch_add(&pl.hdr->next_option, 1u, __ATOMIC_RELAXED, AGENT);
        __syncthreads();
        const ll o = __builtin_amdgcn_readfirstlane(sh.opt);
        __syncthreads();
        if (o >= n) break;
        if (tid == 0 && o < MAX_WG) __hip_atomic_exchange(pl.drivers + o, (int)blockIdx.x, __ATOMIC_RELAXED, AGENT);
        const Desc d = descs[o];
        if (d.model < 0) {  // rejected on the host: no work, price NaN
            if (tid == 0) {
                price[d.out_index] = NAN;
                if (err) err[d.out_index] = DEV_OK;
                stats[d.out_index] = Stats{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
                __hip_atomic_fetch_add((unsigned long long *)&pl.hdr->status, 1ull, __ATOMIC_RELEASE, AGENT);
            }
        } else {
            drive_option<PREC>(d, o, ws, tw, price, bnd, bnd_stride, err, stats, pl, tn, lds, twl, twf, stk, &sp_sh, &err_sh,
                         &ret_sh, &leaf_sh, red_sh, &val_sh, &st_sh, &sh);
        }
        __syncthreads();
    }
    helper_loop<PREC>(pl, n, descs, ws, &sh, lds, tw, twl, twf, tn.idle_ticks);
}

// Clears the pool header, the summary bitmap and the slot words before a
// launch, and sets every job slot's control word to "done" with zero counts.
// A helper may see a slot's flag before the owner's store of the slot's new
// control word (the flag is set after it, without ordering), and its claim
// then lands on the previous value: within a launch that is a finished job,
// on which a claim fails; before a slot's first job it must be one as well,
// not whatever the workspace held.  The solve kernel reads these words only
// with atomic read-modify-writes, so they are written with atomic exchanges:
// the writes must be visible to those atomics even where consecutive kernels
// of a captured graph run without the cache maintenance separate launches get.
__global__ void pool_init_kernel(PoolHdr *hdr, unsigned long long *summary, unsigned long long *bits, int *drivers,
                                 Job *jobs, int n_wg)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long *h64 = (unsigned long long *)hdr;
    if (t == 0) __hip_atomic_exchange(h64, (unsigned long long)(unsigned)n_wg << 32, __ATOMIC_RELAXED, AGENT);
    else if (t < 16) __hip_atomic_exchange(h64 + t, 0ull, __ATOMIC_RELAXED, AGENT);
    if (t < MAX_WG / 64) __hip_atomic_exchange(summary + t, 0ull, __ATOMIC_RELAXED, AGENT);
    if (t < n_wg) __hip_atomic_exchange(bits + t, 0ull, __ATOMIC_RELAXED, AGENT);
    if (t < MAX_WG) __hip_atomic_exchange(drivers + t, -1, __ATOMIC_RELAXED, AGENT);
    if (t < n_wg * JPW) {
        Job *jb = jobs + t;
        __hip_atomic_exchange(&jb->ctl, mkctl(0, PH_DONE, 0, 0), __ATOMIC_RELAXED, AGENT);
        for (int k = 0; k < 3; ++k) __hip_atomic_exchange(&jb->done[k], 0u, __ATOMIC_RELAXED, AGENT);
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

int launch_solve(const Desc *d_desc, int64_t n, char *d_ws, const void *d_tw, double *d_price, int64_t *d_bnd,
                 int64_t bnd_stride, int32_t *d_err, const Tune &tune, void *stream)
{
    if (n <= 0) return 0;
    int n_wg = tune.workgroups;
    if (n_wg < 1 || n_wg > MAX_WG) return 1;
    char *pool = d_ws + pool_offset(n);
    Pool pl;
    pl.hdr = (PoolHdr *)pool;
    pl.summary = (unsigned long long *)(pool + POOL_SUMMARY);
    pl.bits = (unsigned long long *)(pool + POOL_BITS);
    pl.jobs = (Job *)(pool + POOL_JOBS);
    pl.drivers = (int *)(pool + POOL_DRV);
    pl.n_wg = n_wg;
    const int n_init = n_wg * JPW > MAX_WG ? n_wg * JPW : MAX_WG;  // threads: job slots, driver entries
    hipLaunchKernelGGL(pool_init_kernel, dim3((unsigned)((n_init + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       pl.hdr, pl.summary, pl.bits, pl.drivers, pl.jobs, n_wg);
    auto kern = tune.prec ? solve_kernel<1> : solve_kernel<0>;
    if (!d_err) d_err = (int32_t *)(d_ws + err_offset(n));
    Tune tn = tune;
    tn.late_after = (int32_t)(((int64_t)tune.late_after * n + 99) / 100);  // percentage -> options
    hipLaunchKernelGGL(kern, dim3((unsigned)n_wg), dim3(WG), 0, (hipStream_t)stream, d_desc, (ll)n, d_ws,
                       (const double2 *)d_tw, d_price, (ll *)d_bnd, (ll)bnd_stride, d_err,
                       (Stats *)(d_ws + stats_offset(n)), pl, tn);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

}  // namespace aop
