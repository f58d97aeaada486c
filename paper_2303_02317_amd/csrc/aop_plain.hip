// aop_plain.hip -- the plain Theta(T^2) backward induction of Fig. 1 on gfx950,
// batched over options: the comparison path for the FFT method.
//
// Every cell of the lattice / grid is updated with the direct
// max(continuation, exercise) stencil, in FP64, with the tie rule of
// Definition 2.1.  Temporal tiling: one launch advances every option by R
// rows; each wave64 holds a tile of 64*C consecutive cells in registers
// (C per lane), takes the R row steps with neighbour values exchanged by
// wave shuffles, and writes back the cells whose dependency cone stayed inside
// the tile (R*span cells of halo are recomputed by the neighbouring tile).
// Exercise values are carried per cell by one multiplication per row and
// re-seeded with exp() at every launch.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <math.h>
#include <stdint.h>

#include "aop_internal.h"

namespace aop {

typedef long long ll;

#define PL_C 16                    // cells per lane
#define PL_W (64 * PL_C)           // cells per wave tile
#define PL_R 64                    // rows per launch
#define PL_WAVES 4                 // waves (tiles) per workgroup

__device__ __forceinline__ bool pl_red(double c, double e)
{
    return (c >= e) && (c < INFINITY) && (e < INFINITY);
}

// Largest v over the wave's lanes (uniform result).
__device__ __forceinline__ ll wave_max(ll v)
{
    for (int o = 32; o >= 1; o >>= 1) {
        const ll w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

// Record a tile's candidate for a row's boundary: the row's boundary is the
// largest candidate over the tiles (every cell of the row is computed, with
// its whole dependency cone, by at least one tile).
__device__ __forceinline__ void note_boundary(ll *row, ll v)
{
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0 && v > LLONG_MIN)
        __hip_atomic_fetch_max(row, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Boundary rows start at "none": -1 (lattices) or INT64_MIN (BSM).
__global__ void plain_bnd_init(const Desc *__restrict__ descs, ll *bnd, ll stride)
{
    const Desc d = descs[blockIdx.y];
    const ll none = d.model == BSM ? LLONG_MIN : -1;
    for (ll i = (ll)blockIdx.x * blockDim.x + threadIdx.x; i < stride; i += (ll)gridDim.x * blockDim.x)
        bnd[(ll)blockIdx.y * stride + i] = none;
}

// One launch: option blockIdx.y, tiles blockIdx.x * PL_WAVES + wave.
// Lattices: rows itop -> itop - r (r = min(R, itop)), itop = T - L*R, the
// input row of the first launch (row T) evaluated in closed form.
// BSM: steps n -> n + r, n = L*R, r = min(R, T - n), step 0 in closed form.
// BND: also record each row's boundary (kept out of the loop when not asked for).
template <bool BND>
__global__ void __launch_bounds__(64 * PL_WAVES) plain_kernel(const Desc *__restrict__ descs, char *ws,
                                                              double *price, ll L, ll *bnd_all, ll stride)
{
    const Desc d = descs[blockIdx.y];
    if (d.model < 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && L == 0) price[d.out_index] = NAN;
        return;
    }
    const ll T = d.T;
    const int lane = threadIdx.x & 63;
    const ll tile = (ll)blockIdx.x * PL_WAVES + (threadIdx.x >> 6);
    double *rowA = (double *)(ws + d.ws_off);
    double *rowB = rowA + d.row_len;
    double *in = (L & 1) ? rowB : rowA;
    double *out = (L & 1) ? rowA : rowB;
    ll *bnd = BND ? bnd_all + (ll)blockIdx.y * stride : nullptr;
    double g[PL_C], x[PL_C];

    if (d.model != BSM) {
        const bool bin = d.model == BINOMIAL;
        const int span = bin ? 1 : 2;
        const ll itop = T - L * PL_R;
        if (itop <= 0) return;
        const ll r = itop < PL_R ? itop : PL_R;
        const ll wout = PL_W - span * r;           // valid cells per tile
        const ll ilast = bin ? itop : 2 * itop;     // last column of row itop
        const ll j0 = tile * wout;
        if (j0 > (bin ? itop - r : 2 * (itop - r))) return;
        const double u = exp(d.a);
        for (int c = 0; c < PL_C; ++c) {
            const ll j = j0 + lane * PL_C + c;
            const double ex = d.S * exp((double)((bin ? 2 * j : j) - itop) * d.a);
            x[c] = ex;
            if (L == 0) {
                const double e = ex - d.K;
                g[c] = (j <= ilast) ? (pl_red(0.0, e) ? 0.0 : e) : 0.0;
            } else {
                g[c] = (j <= ilast) ? in[j] : 0.0;
            }
        }
        if (BND && L == 0) {  // expiry row: red = out of the money
            ll last = LLONG_MIN;
            for (int c = 0; c < PL_C; ++c) {
                const ll j = j0 + lane * PL_C + c;
                if (j <= ilast && pl_red(0.0, x[c] - d.K)) last = j;
            }
            note_boundary(bnd + itop, last);
        }
        for (ll k = 1; k <= r; ++k) {
            const double n0 = __shfl_down(g[0], 1, 64);
            const double n1 = __shfl_down(g[1], 1, 64);
            double nx[PL_C];
            if (bin) {
#pragma unroll
                for (int c = 0; c < PL_C - 1; ++c) nx[c] = d.w0 * g[c] + d.w1 * g[c + 1];
                nx[PL_C - 1] = d.w0 * g[PL_C - 1] + d.w1 * n0;
            } else {
#pragma unroll
                for (int c = 0; c < PL_C - 2; ++c) nx[c] = d.w0 * g[c] + d.w1 * g[c + 1] + d.w2 * g[c + 2];
                nx[PL_C - 2] = d.w0 * g[PL_C - 2] + d.w1 * g[PL_C - 1] + d.w2 * n0;
                nx[PL_C - 1] = d.w0 * g[PL_C - 1] + d.w1 * n0 + d.w2 * n1;
            }
            const bool ex = exercise_row(d, itop - k);  // uniform
            if (BND) {
                ll last = LLONG_MIN;
                const ll irow = itop - k;
#pragma unroll
                for (int c = 0; c < PL_C; ++c) {
                    x[c] *= u;  // S u^{col - i} one row lower
                    const double e = x[c] - d.K;
                    const bool red = !ex || pl_red(nx[c], e);
                    g[c] = red ? nx[c] : e;
                    // a cell is exact where its cone stayed inside the tile
                    const ll loc = lane * PL_C + c;
                    if (red && loc < PL_W - span * k && j0 + loc <= (bin ? irow : 2 * irow)) last = j0 + loc;
                }
                if (d.ex_every != 0) note_boundary(bnd + irow, ex ? last : (bin ? irow : 2 * irow));
            } else {
#pragma unroll
                for (int c = 0; c < PL_C; ++c) {
                    x[c] *= u;  // S u^{col - i} one row lower
                    const double e = x[c] - d.K;
                    g[c] = (!ex || pl_red(nx[c], e)) ? nx[c] : e;
                }
            }
        }
        const ll iout = itop - r;
        const ll olast = bin ? iout : 2 * iout;
        for (int c = 0; c < PL_C; ++c) {
            const ll loc = lane * PL_C + c;
            const ll j = j0 + loc;
            if (loc < wout && j <= olast) out[j] = g[c];
        }
        if (iout == 0 && j0 == 0 && lane == 0) price[d.out_index] = g[0];
    } else {
        const ll n = L * PL_R;
        if (n >= T) return;
        const ll r = (T - n) < PL_R ? (T - n) : PL_R;
        const ll wout = PL_W - 2 * r;
        const ll lo_out = -(T - n - r);            // cone of step n + r
        const ll k0 = lo_out + tile * wout;        // first output cell of this tile
        if (k0 > T - n - r) return;
        const ll kb = k0 - r;                      // first input cell
        double *A = in + 2 * T + 1, *B = out + 2 * T + 1;
        for (int c = 0; c < PL_C; ++c) {
            const ll k = kb + lane * PL_C + c;
            const double gk = 1.0 - exp(d.s0 + (double)k * d.a);
            x[c] = gk;
            const bool incone = (k >= -(T - n)) && (k <= T - n);
            if (L == 0)
                g[c] = gk > 0.0 ? gk : 0.0;
            else
                g[c] = incone ? A[k] : 0.0;
        }
        if (BND && L == 0) {  // expiry step: exercise where the payoff is positive
            ll last = LLONG_MIN;
            for (int c = 0; c < PL_C; ++c) {
                const ll k = kb + lane * PL_C + c;
                if (k <= T && k >= -T && x[c] > 0.0) last = k;  // closed form: every cell is exact
            }
            note_boundary(bnd, last);
        }
        for (ll k = 1; k <= r; ++k) {
            const double pv = __shfl_up(g[PL_C - 1], 1, 64);
            const double nv = __shfl_down(g[0], 1, 64);
            double nx[PL_C];
            nx[0] = d.w0 * pv + d.w1 * g[0] + d.w2 * g[1];
#pragma unroll
            for (int c = 1; c < PL_C - 1; ++c) nx[c] = d.w0 * g[c - 1] + d.w1 * g[c] + d.w2 * g[c + 1];
            nx[PL_C - 1] = d.w0 * g[PL_C - 2] + d.w1 * g[PL_C - 1] + d.w2 * nv;
            if (BND) {
                ll last = LLONG_MIN;
                const ll hw = T - n - k;  // cone of step n + k: |cell| <= hw
#pragma unroll
                for (int c = 0; c < PL_C; ++c) {
                    const bool green = d.ex_every != 0 && x[c] > nx[c];
                    g[c] = green ? x[c] : nx[c];
                    const ll loc = lane * PL_C + c;
                    const ll kk = kb + loc;
                    if (green && loc >= k && loc < PL_W - k && kk >= -hw && kk <= hw) last = kk;
                }
                if (d.ex_every != 0) note_boundary(bnd + n + k, last);
            } else {
#pragma unroll
                for (int c = 0; c < PL_C; ++c) g[c] = (d.ex_every != 0 && x[c] > nx[c]) ? x[c] : nx[c];
            }
        }
        const ll hi_out = T - n - r;
        for (int c = 0; c < PL_C; ++c) {
            const ll loc = lane * PL_C + c;
            const ll k = kb + loc;
            if (loc >= r && loc < r + wout && k <= hi_out) B[k] = g[c];
            if (n + r == T && k == 0 && loc >= r && loc < r + wout) price[d.out_index] = d.K * g[c];
        }
    }
}

// Host loop: ceil(Tmax / R) launches; grid.x covers the widest option's tiles.
int launch_plain_batch(const Desc *d_desc, const Desc *h_desc, int64_t n, char *d_ws, double *d_price,
                       int64_t *d_bnd, int64_t bnd_stride, void *stream)
{
    if (n <= 0) return 0;
    if (d_bnd) {
        hipLaunchKernelGGL(plain_bnd_init, dim3(64, (unsigned)n), dim3(256), 0, (hipStream_t)stream, d_desc,
                           (ll *)d_bnd, (ll)bnd_stride);
        if (hipGetLastError() != hipSuccess) return 1;
    }
    ll Tmax = 0;
    int span = 1;
    for (int64_t i = 0; i < n; ++i)
        if (h_desc[i].model >= 0) {
            Tmax = h_desc[i].T > Tmax ? h_desc[i].T : Tmax;
            if (h_desc[i].model != BINOMIAL) span = 2;
        }
    const ll launches = Tmax > 0 ? (Tmax + PL_R - 1) / PL_R : 1;
    for (ll L = 0; L < launches; ++L) {
        // widest row among options at this launch
        ll width = 1;
        for (int64_t i = 0; i < n; ++i) {
            const Desc &d = h_desc[i];
            if (d.model < 0) continue;
            ll w;
            if (d.model == BSM) w = 2 * (d.T - L * PL_R) + 1;
            else w = (d.model == BINOMIAL ? 1 : 2) * (d.T - L * PL_R) + 1;
            width = w > width ? w : width;
        }
        const ll wout = PL_W - span * PL_R;
        const ll tiles = (width + wout - 1) / wout + 1;
        const unsigned gx = (unsigned)((tiles + PL_WAVES - 1) / PL_WAVES);
        if (d_bnd)
            hipLaunchKernelGGL(plain_kernel<true>, dim3(gx, (unsigned)n), dim3(64 * PL_WAVES), 0, (hipStream_t)stream,
                               d_desc, d_ws, d_price, L, (ll *)d_bnd, (ll)bnd_stride);
        else
            hipLaunchKernelGGL(plain_kernel<false>, dim3(gx, (unsigned)n), dim3(64 * PL_WAVES), 0,
                               (hipStream_t)stream, d_desc, d_ws, d_price, L, (ll *)nullptr, (ll)0);
        if (hipGetLastError() != hipSuccess) return 1;
    }
    return 0;
}

}  // namespace aop
