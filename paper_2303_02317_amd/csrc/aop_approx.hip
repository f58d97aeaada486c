// aop_approx.hip -- Gaussian approximations of the European binomial call
// (the paper's section on the European call under the binomial model): the
// number of up moves x of the T-step lattice is replaced by a normal variable
// with mean pT and variance v = p(1-p)T,
//   price ~ m^T / sqrt(2 pi v) * sum_x (S u^{2x-T} - K)^+ e^{-(x - pT)^2 / (2v)},
// summed over a window of 6 standard deviations (O(sqrt T) terms) or over
// x in [0, T-1] (O(T) terms), or integrated over x in closed form with erf
// (O(1)).  One workgroup per option; the sums are FP64 with a workgroup
// reduction.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "aop_internal.h"

namespace aop {

typedef long long ll;

#define AP_WG 256

__global__ void __launch_bounds__(AP_WG) approx_kernel(const ApproxParam *__restrict__ prm, ll n, double *price)
{
    __shared__ double part[AP_WG / 64];
    const ll o = blockIdx.x;
    if (o >= n) return;
    const ApproxParam q = prm[o];
    const int tid = threadIdx.x;
    if (!q.valid) {
        if (tid == 0) price[o] = NAN;
        return;
    }
    const double T = (double)q.T;
    if (q.method == 2) {
        if (tid == 0) {
            // integral of (S u^{2x-T} - K) N(x; pT, v) dx from x0 = ceil(T/2 + ln(K/S)/(2 ln u)) to T:
            // completing the square, e^{2 a x} N(x; mu, v) = e^{2 a mu + 2 a^2 v} N(x; mu + 2 a v, v)
            const double a = q.a, mu = q.mu, v = q.v;
            double lo = ceil(0.5 * T + log(q.K / q.S) / (2.0 * a));
            lo = lo > T ? T : lo;
            const double sv2 = sqrt(2.0 * v);
            const double gS = q.S * exp((2.0 * (v * a + mu) - T) * a);
            const double sterm = gS * (erf((T - mu) / sv2 - a * sv2) - erf((lo - mu) / sv2 - a * sv2));
            const double kterm = q.K * (erf((T - mu) / sv2) - erf((lo - mu) / sv2));
            price[o] = 0.5 * q.disc * (sterm - kterm);
        }
        return;
    }
    double acc = 0.0;
    const double inv2v = 1.0 / (2.0 * q.v);
    for (ll x = q.xlo + tid; x <= q.xhi; x += AP_WG) {
        const double pay = q.S * exp((double)(2 * x - q.T) * q.a) - q.K;
        const double dx = (double)x - q.mu;
        if (pay > 0.0) acc += pay * exp(-dx * dx * inv2v);
    }
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((tid & 63) == 0) part[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < AP_WG / 64; ++w) s += part[w];
        price[o] = q.disc * s / sqrt(2.0 * M_PI * q.v);
    }
}

int launch_approx(const ApproxParam *d_prm, int64_t n, double *d_price, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(approx_kernel, dim3((unsigned)n), dim3(AP_WG), 0, (hipStream_t)stream, d_prm, (ll)n, d_price);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

}  // namespace aop
