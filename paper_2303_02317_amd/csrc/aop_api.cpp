// aop_api.cpp -- host side of libaop's C ABI (declared in include/aop.h).
//
// Validates options, derives the lattice / grid parameters from the paper's
// formulas (Fig. 1 and Sec. 2.1 for the binomial lattice, Sec. 3 for the
// trinomial lattice, eq. (bsmG) of Sec. 4.2 for the BSM grid), lays out the
// caller's device workspace and launches the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "aop.h"
#include "aop_host.h"
#include "aop_internal.h"

using aop::Desc;

namespace {

inline size_t align_up(size_t x) { return aop::ws_align(x); }
inline int64_t next_pow2(int64_t n)
{
    int64_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

// Fill the model parameters of a descriptor; returns an aop_status.
aop_status make_desc(const aop_option &o, double lambda, Desc &d)
{
    std::memset(&d, 0, sizeof(d));
    d.model = -1;
    if (!(std::isfinite(o.S0) && std::isfinite(o.K) && std::isfinite(o.r) && std::isfinite(o.q) &&
          std::isfinite(o.sigma) && std::isfinite(o.expiry)))
        return AOP_EINVAL;
    if (o.S0 <= 0 || o.K <= 0 || o.sigma <= 0 || o.expiry <= 0 || o.q < 0 || o.T < 1 ||
        (o.flags & ~AOP_EUROPEAN) != 0)
        return AOP_EINVAL;
    const bool european = (o.flags & AOP_EUROPEAN) != 0;
    if (o.exercise_every < 0 || (european && o.exercise_every > 1)) return AOP_EINVAL;
    if (o.exercise_every > 1 && o.model != AOP_BINOMIAL_CALL) return AOP_ENOTIMPL;
    if (o.T > AOP_MAX_T) return AOP_ETOOBIG;
    const double T = (double)o.T;
    d.T = o.T;
    d.S = o.S0;
    d.K = o.K;
    switch (o.model) {
    case AOP_BINOMIAL_CALL: {
        // Fig. 1: dt = E/T, u = e^{V sqrt(dt)}, d = 1/u, p = (e^{(R-Y)dt} - d)/(u - d), m = e^{-R dt};
        // Sec. 2.1: s0 = m(1-p) on the down child G[i+1][j], s1 = mp on the up child G[i+1][j+1].
        const double dt = o.expiry / T;
        const double a = o.sigma * std::sqrt(dt);
        const double u = std::exp(a), dn = 1.0 / u;
        const double p = (std::exp((o.r - o.q) * dt) - dn) / (u - dn);
        const double m = std::exp(-o.r * dt);
        if (!(p > 0.0 && p < 1.0)) return AOP_EPROB;
        d.a = a;
        // Lemma 2.3: with Y = 0 and R >= 0 no cell below the expiry row
        // exercises; with R < 0 exercise can pay deep in the money.
        d.no_green = (o.q == 0.0 && o.r >= 0.0);
        d.w0 = m * (1.0 - p);
        d.w1 = m * p;
        d.w2 = 0.0;
        break;
    }
    case AOP_TRINOMIAL_CALL: {
        // Sec. 3: u = e^{V sqrt(2 dt)}, p_u = ((e^{(R-Y)dt/2} - sqrt d)/(sqrt u - sqrt d))^2,
        // p_d = ((sqrt u - e^{(R-Y)dt/2})/(sqrt u - sqrt d))^2, p_o = 1 - p_u - p_d;
        // children j (down, m p_d), j+1 (same, m p_o), j+2 (up, m p_u).
        const double dt = o.expiry / T;
        const double A = o.sigma * std::sqrt(2.0 * dt);
        const double su = std::exp(0.5 * A), sd = std::exp(-0.5 * A);
        const double g = std::exp(0.5 * (o.r - o.q) * dt);
        const double pu = ((g - sd) / (su - sd)) * ((g - sd) / (su - sd));
        const double pd = ((su - g) / (su - sd)) * ((su - g) / (su - sd));
        const double po = 1.0 - pu - pd;
        const double m = std::exp(-o.r * dt);
        if (!(pu > 0.0 && pd > 0.0 && po >= 0.0)) return AOP_EPROB;
        // The trinomial boundary lemmas of Sec. 3 (the boundary drops by at
        // most two columns per row, so a trapezoid's left part is all
        // continuation) are shown for a non-negative risk-free rate.  With
        // R < 0 and no dividend a row's top cell can exercise under an
        // all-continuation row, a drop of three or more columns, so the
        // decomposition does not apply.
        if (o.r < 0.0 && !european) return AOP_EPROB;  // (American trinomial only)
        d.a = A;
        d.no_green = (o.q == 0.0 && o.r >= 0.0);  // as for the binomial lattice
        d.w0 = m * pd;
        d.w1 = m * po;
        d.w2 = m * pu;
        break;
    }
    case AOP_BSM_PUT: {
        // Sec. 4.2: s = ln(x/K), tau = sigma^2 (E - t)/2, omega = 2R/sigma^2; eq. (bsmG):
        // v^{n+1}_k = (1 - omega dtau - 2 dtau/ds^2) v_k + sum_{h=+-1} (dtau/ds^2 + h (omega-1)/2 dtau/ds) v_{k+h}.
        if (o.q != 0.0) return AOP_EINVAL;
        if (!(lambda > 0.0 && lambda <= 0.5)) return AOP_EINVAL;
        const double dtau = 0.5 * o.sigma * o.sigma * o.expiry / T;
        const double ds = std::sqrt(dtau / lambda);
        const double omega = 2.0 * o.r / (o.sigma * o.sigma);
        const double lam = dtau / (ds * ds);
        const double drift = 0.5 * (omega - 1.0) * dtau / ds;
        const double ca = lam + drift, cb = lam - drift, cc = 1.0 - omega * dtau - 2.0 * lam;
        if (!(ca >= 0.0 && cb >= 0.0 && cc >= 0.0)) return AOP_EPROB;
        d.a = ds;
        d.s0 = std::log(o.S0 / o.K);
        d.w0 = cb;  // k-1
        d.w1 = cc;  // k
        d.w2 = ca;  // k+1
        break;
    }
    default:
        return AOP_EINVAL;
    }
    d.model = o.model;
    d.ex_every = european ? 0 : (o.exercise_every > 1 ? (int32_t)std::min<int64_t>(o.exercise_every, o.T + 1) : 1);
    return AOP_OK;
}

// Per-option workspace geometry (doubles / complex elements).
void geometry(Desc &d)
{
    const int64_t T = d.T;
    int64_t nin_max;
    if (d.model == aop::BINOMIAL) {
        d.row_len = T + 2;
        d.arena_len = 2 * d.row_len + 256;
        nin_max = T;
    } else if (d.model == aop::TRINOMIAL) {
        d.row_len = 2 * T + 3;
        d.arena_len = 2 * d.row_len + 256;
        nin_max = 2 * T + 1;
    } else {
        d.row_len = 3 * T + 3;  // k in [-2T-1, T+1]
        d.arena_len = 4 * T + 256;
        nin_max = 2 * T + 1;
    }
    d.nfft = std::max<int64_t>(next_pow2(std::max<int64_t>(nin_max, 2)), 2);
    // The correlations a driver has in flight at once use the scratch as a
    // stack: one per recursion depth, each at most half the size of its
    // parent's, plus (BSM) the top-level correlation beside the trapezoid.
    d.scr_len = 4 * d.nfft;
}

size_t option_bytes(const Desc &d)
{
    return align_up(sizeof(double) * (size_t)(2 * d.row_len + d.arena_len)) + align_up(16 * (size_t)d.scr_len) +
           align_up(16 * (size_t)aop::SPC_E * (size_t)aop::spc_entry(d.nfft));
}

// Descriptors for the plain stencil: two row buffers per option.
size_t build_plain(const aop_option *opts, int64_t n, double lambda, Desc *out, int32_t *status)
{
    size_t off = align_up(sizeof(Desc) * (size_t)std::max<int64_t>(n, 1));
    for (int64_t i = 0; i < n; ++i) {
        Desc &d = out[i];
        aop_status st = make_desc(opts[i], lambda, d);
        d.out_index = i;
        if (status) status[i] = st;
        if (st != AOP_OK) {
            d.model = -1;
            continue;
        }
        geometry(d);
        d.ws_off = (int64_t)off;
        off += align_up(sizeof(double) * 2 * (size_t)d.row_len);
    }
    return off;
}

// Estimated solve cost of an option (work ~ T log^2 T; the trinomial and BSM
// rows are twice as long), used to hand out the largest options first.
static double option_cost(const Desc &d)
{
    if (d.model < 0) return -1.0;
    const double T = (double)d.T, lg = std::log2(T + 1.0);
    return (d.model == aop::BINOMIAL ? 1.0 : 2.0) * T * (lg * lg + 1.0);
}

// Build descriptors for a batch; returns total workspace bytes.  Descriptors
// are stored in decreasing order of estimated cost (the order in which the
// persistent kernel's workgroups claim them); out_index keeps each option's
// position in the caller's arrays.

// Descriptors of a batch built straight into `out` (n entries) without any
// heap allocation: stable insertion sort by decreasing cost (small n only).
size_t build_batch_in_place(const aop_option *opts, int64_t n, int32_t prec, double lambda, Desc *out,
                            int32_t *status)
{
    for (int64_t i = 0; i < n; ++i) {
        Desc &d = out[i];
        aop_status st = make_desc(opts[i], lambda, d);
        if (st == AOP_OK && prec != AOP_FP64 && prec != AOP_MIXED) st = AOP_EINVAL;
        d.out_index = i;
        d.prec = prec;
        if (status) status[i] = st;
        if (st != AOP_OK) {
            d.model = -1;
            continue;
        }
        geometry(d);
    }
    for (int64_t i = 1; i < n; ++i) {
        const Desc x = out[i];
        const double cx = option_cost(x);
        int64_t k = i;
        while (k > 0 && option_cost(out[k - 1]) < cx) {
            out[k] = out[k - 1];
            --k;
        }
        out[k] = x;
    }
    size_t off = (size_t)aop::options_offset(n);
    for (int64_t k = 0; k < n; ++k)
        if (out[k].model >= 0) {
            out[k].ws_off = (int64_t)off;
            off += option_bytes(out[k]);
        }
    return off;
}

// Workspace of aop_price_batch_noalloc: a fixed device array, one per GPU.
// Host code never passes `scratch` itself to a kernel or copy: its address on
// each device comes from hipGetSymbolAddress, taken once per device when a
// context is created there (with that device current).
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(256) << 20;
constexpr int64_t NOALLOC_MAX_OPTIONS = 256;
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES];
}  // namespace

static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
// With `device` current: resolve this device's copy of `scratch` (once).
aop_status scratch_setup(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return AOP_EINVAL;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr[device]) return AOP_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return AOP_EDEVICE;
    g_scratch_ptr[device] = ptr;
    return AOP_OK;
}

void *scratch_of(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    return g_scratch_ptr[device];
}
}  // namespace

namespace aop {

size_t build_batch(const aop_option *opts, int64_t n, int32_t prec, double lambda, Desc *out, int32_t *status)
{
    std::vector<Desc> tmp((size_t)std::max<int64_t>(n, 1));
    for (int64_t i = 0; i < n; ++i) {
        Desc &d = tmp[(size_t)i];
        aop_status st = make_desc(opts[i], lambda, d);
        if (st == AOP_OK && prec != AOP_FP64 && prec != AOP_MIXED) st = AOP_EINVAL;
        d.out_index = i;
        d.prec = prec;
        if (status) status[i] = st;
        if (st != AOP_OK) {
            d.model = -1;
            continue;
        }
        geometry(d);
    }
    std::vector<int64_t> order((size_t)std::max<int64_t>(n, 0));
    for (int64_t i = 0; i < n; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        return option_cost(tmp[(size_t)a]) > option_cost(tmp[(size_t)b]);
    });
    size_t off = (size_t)aop::options_offset(n);
    for (int64_t k = 0; k < n; ++k) {
        Desc d = tmp[(size_t)order[(size_t)k]];
        if (d.model >= 0) {
            d.ws_off = (int64_t)off;
            off += option_bytes(d);
        }
        out[k] = d;
    }
    return off;
}

size_t option_area_bytes(const aop_option &o, double lambda)
{
    Desc d;
    if (make_desc(o, lambda, d) != AOP_OK) return 0;
    geometry(d);
    return option_bytes(d);
}

Tune make_tune(const aop_tuning &t, double tick_hz, int32_t workgroups)
{
    Tune tune;
    tune.workgroups = workgroups > 0 ? std::min(workgroups, MAX_WG) : t.workgroups;
    tune.pub_min_lg = t.pub_min_lg;
    tune.pub_direct = t.pub_direct;
    tune.direct_max_h = t.direct_max_h;
    tune.direct_max_n = t.direct_max_n;
    tune.prec = 0;
    tune.late_pub_lg = t.late_pub_min_lg;
    tune.lds_lg64 = t.lds_max_lg;
    tune.radix = t.radix_lg;
    tune.late_after = t.late_after_pct;  // a percentage until the launch converts it
    tune.timeout_ticks = t.timeout_us > 0 ? (int64_t)(1e-6 * (double)t.timeout_us * tick_hz)
                                          : (int64_t)(1e-3 * (double)t.timeout_ms * tick_hz);
    tune.idle_ticks = (int64_t)(1e-6 * (double)t.helper_idle_us * tick_hz);
    return tune;
}

bool tuning_valid(const aop_tuning &u)
{
    return u.workgroups >= 1 && u.workgroups <= MAX_WG && u.pub_min_lg >= 1 && u.pub_min_lg <= 30 &&
           u.direct_max_h >= 0 && u.direct_max_h <= DIRECT_MAX_H && u.direct_max_n >= 0 && u.direct_max_n <= DIRECT_MAX_N && u.helper_idle_us >= 1 &&
           u.late_pub_min_lg >= 0 && u.late_pub_min_lg <= 30 && u.late_after_pct >= 0 && u.late_after_pct <= 100 &&
           u.timeout_ms > 0 && u.timeout_ms <= 3600000 && u.timeout_us >= 0 && u.timeout_us <= 3600000000ll &&
           (u.lds_max_lg == 11 || u.lds_max_lg == 12) &&
           (u.radix_lg == 2 || u.radix_lg == 3);
}

}  // namespace aop

namespace {

aop_status ensure_stage(aop_ctx *ctx, size_t n)
{
    if (ctx->stage_pending) {
        if (hipEventSynchronize(ctx->stage_done) != hipSuccess) return AOP_EDEVICE;
        ctx->stage_pending = false;
    }
    if (n <= ctx->stage_cap) return AOP_OK;
    if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
    ctx->h_stage = nullptr;
    ctx->stage_cap = 0;
    size_t cap = std::max<size_t>(n, 64);
    if (hipHostMalloc((void **)&ctx->h_stage, cap * sizeof(Desc), hipHostMallocDefault) != hipSuccess)
        return AOP_ENOMEM;
    ctx->stage_cap = cap;
    return AOP_OK;
}

}  // namespace

extern "C" {

const char *aop_version(void) { return "aop-mi355x 0.1 (gfx950)"; }

const char *aop_status_str(aop_status s)
{
    switch (s) {
    case AOP_OK: return "ok";
    case AOP_EINVAL: return "invalid argument";
    case AOP_EPROB: return "lattice probability or scheme coefficient out of range";
    case AOP_ENOMEM: return "out of memory / workspace too small";
    case AOP_EDEVICE: return "HIP device error";
    case AOP_ETOOBIG: return "T above AOP_MAX_T";
    case AOP_ECANCELED: return "canceled";
    case AOP_ENOTIMPL: return "not implemented for this model/precision";
    }
    return "unknown status";
}

size_t aop_twiddle_bytes(void) { return sizeof(double) * 2 * (size_t)aop::TW_N; }

aop_status aop_ctx_create(int device, double lambda, void *d_twiddles, size_t tw_bytes, aop_ctx **out)
{
    if (!out) return AOP_EINVAL;
    *out = nullptr;
    if (lambda == 0.0) lambda = 1.0 / 3.0;
    if (!(lambda > 0.0 && lambda <= 0.5)) return AOP_EINVAL;
    if (!d_twiddles || (reinterpret_cast<uintptr_t>(d_twiddles) & 15u) != 0) return AOP_EINVAL;
    if (tw_bytes < aop_twiddle_bytes()) return AOP_ENOMEM;
    aop_ctx *ctx = new (std::nothrow) aop_ctx;
    if (!ctx) return AOP_ENOMEM;
    ctx->device = device;
    ctx->lambda = lambda;
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return AOP_EDEVICE;
    }
    ctx->d_tw = d_twiddles;  // the caller's memory: filled here, never freed here
    if (scratch_setup(device) != AOP_OK) {
        delete ctx;
        return AOP_EDEVICE;
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || ncu < 1)
        ncu = 1;
    ctx->n_cu = ncu;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
        ctx->tick_hz = 1e3 * (double)khz;
    ctx->tuning.workgroups = std::min(ncu, aop::MAX_WG);
    ctx->tuning.pub_min_lg = 13;
    ctx->tuning.pub_direct = 0;
    ctx->tuning.direct_max_h = 320;
    ctx->tuning.direct_max_n = 2048;
    ctx->tuning.helper_idle_us = 20000;
    ctx->tuning.late_pub_min_lg = 10;
    ctx->tuning.late_after_pct = 50;
    ctx->tuning.timeout_ms = 30000;
    ctx->tuning.timeout_us = 0;
    ctx->tuning.lds_max_lg = 12;
    ctx->tuning.radix_lg = 3;
    if (hipEventCreateWithFlags(&ctx->stage_done, hipEventDisableTiming) != hipSuccess ||
        aop::launch_twiddles(ctx->d_tw, nullptr) != 0 || hipDeviceSynchronize() != hipSuccess) {
        if (ctx->stage_done) (void)hipEventDestroy(ctx->stage_done);
        delete ctx;
        return AOP_EDEVICE;
    }
    // descriptor staging sized for aop_price_batch_noalloc, which must not allocate
    if (ensure_stage(ctx, (size_t)NOALLOC_MAX_OPTIONS) != AOP_OK) {
        (void)hipEventDestroy(ctx->stage_done);
        delete ctx;
        return AOP_ENOMEM;
    }
    *out = ctx;
    return AOP_OK;
}

aop_status aop_ctx_destroy(aop_ctx *ctx)
{
    if (!ctx) return AOP_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (ctx->stage_pending) (void)hipEventSynchronize(ctx->stage_done);
    if (ctx->stage_done) (void)hipEventDestroy(ctx->stage_done);
    if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
    delete ctx;  // the twiddle table belongs to the caller
    return AOP_OK;
}

aop_status aop_validate(const aop_option *o, double lambda)
{
    if (!o) return AOP_EINVAL;
    if (lambda == 0.0) lambda = 1.0 / 3.0;
    Desc d;
    return make_desc(*o, lambda, d);
}

aop_status aop_workspace_bytes(const aop_option *opts, int64_t n, int32_t precision, size_t *bytes)
{
    if (!bytes || n < 0 || (n > 0 && !opts)) return AOP_EINVAL;
    std::vector<Desc> d((size_t)std::max<int64_t>(n, 1));
    *bytes = aop::build_batch(opts, n, precision, 1.0 / 3.0, d.data(), nullptr);
    return AOP_OK;
}

aop_status aop_price_batch(aop_ctx *ctx, const aop_option *opts, int64_t n, int32_t precision,
                           void *d_ws, size_t ws_bytes, double *d_price, int32_t *h_status,
                           int64_t *d_bnd, int64_t bnd_stride, void *stream)
{
    if (!ctx || n < 0 || (n > 0 && (!opts || !d_ws || !d_price))) return AOP_EINVAL;
    if (n == 0) return AOP_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return AOP_EDEVICE;
    aop_status st = ensure_stage(ctx, (size_t)n);
    if (st != AOP_OK) return st;
    std::vector<int32_t> stat((size_t)n);
    const size_t need = aop::build_batch(opts, n, precision, ctx->lambda, ctx->h_stage, stat.data());
    if (h_status) std::memcpy(h_status, stat.data(), sizeof(int32_t) * (size_t)n);
    if (ws_bytes < need) return AOP_ENOMEM;
    if (d_bnd) {
        int64_t tmax = 0;
        for (int64_t i = 0; i < n; ++i) tmax = std::max<int64_t>(tmax, opts[i].T);
        if (bnd_stride < tmax + 1) return AOP_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(d_ws, ctx->h_stage, sizeof(Desc) * (size_t)n, hipMemcpyHostToDevice, s) != hipSuccess)
        return AOP_EDEVICE;
    if (hipEventRecord(ctx->stage_done, s) != hipSuccess) return AOP_EDEVICE;
    ctx->stage_pending = true;
    aop::Tune tune = aop::make_tune(*ctx, 0);
    tune.prec = precision;
    if (aop::launch_solve((const Desc *)d_ws, n, (char *)d_ws, ctx->d_tw, d_price, d_bnd, bnd_stride, nullptr, tune,
                          stream) != 0)
        return AOP_EDEVICE;
    return AOP_OK;
}

aop_status aop_price_batch_noalloc(aop_ctx *ctx, const aop_option *opts, int64_t n, int32_t precision,
                                   double *d_price, int32_t *h_status, int64_t *d_bnd, int64_t bnd_stride,
                                   void *stream)
{
    if (!ctx || n < 0 || (n > 0 && (!opts || !d_price))) return AOP_EINVAL;
    if (n == 0) return AOP_OK;
    if (n > NOALLOC_MAX_OPTIONS || ctx->stage_cap < (size_t)n) return AOP_ENOMEM;
    if (hipSetDevice(ctx->device) != hipSuccess) return AOP_EDEVICE;
    char *ws = (char *)scratch_of(ctx->device);
    if (!ws) return AOP_EDEVICE;
    if (ctx->stage_pending) {  // the staging buffer's previous copy must have left it
        if (hipEventSynchronize(ctx->stage_done) != hipSuccess) return AOP_EDEVICE;
        ctx->stage_pending = false;
    }
    int32_t st_local[NOALLOC_MAX_OPTIONS];
    int32_t *st = h_status ? h_status : st_local;
    const size_t need = build_batch_in_place(opts, n, precision, ctx->lambda, ctx->h_stage, st);
    if (need > NOALLOC_SCRATCH_BYTES) return AOP_ENOMEM;
    if (d_bnd) {
        int64_t tmax = 0;
        for (int64_t i = 0; i < n; ++i) tmax = std::max<int64_t>(tmax, opts[i].T);
        if (bnd_stride < tmax + 1) return AOP_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(ws, ctx->h_stage, sizeof(Desc) * (size_t)n, hipMemcpyHostToDevice, s) != hipSuccess)
        return AOP_EDEVICE;
    if (hipEventRecord(ctx->stage_done, s) != hipSuccess) return AOP_EDEVICE;
    ctx->stage_pending = true;
    aop::Tune tune = aop::make_tune(*ctx, 0);
    tune.prec = precision;
    if (aop::launch_solve((const Desc *)ws, n, ws, ctx->d_tw, d_price, d_bnd, bnd_stride, nullptr, tune, stream) != 0)
        return AOP_EDEVICE;
    return AOP_OK;
}

size_t aop_noalloc_scratch_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

size_t aop_approx_workspace_bytes(int64_t n) { return align_up(sizeof(aop::ApproxParam) * (size_t)std::max<int64_t>(n, 1)); }

aop_status aop_european_approx(aop_ctx *ctx, const aop_option *opts, int64_t n, int32_t method, void *d_ws,
                               size_t ws_bytes, double *d_price, int32_t *h_status, void *stream)
{
    if (!ctx || n < 0 || (n > 0 && (!opts || !d_ws || !d_price)) || method < 0 || method > 2) return AOP_EINVAL;
    if (n == 0) return AOP_OK;
    if (ws_bytes < aop_approx_workspace_bytes(n)) return AOP_ENOMEM;
    if (hipSetDevice(ctx->device) != hipSuccess) return AOP_EDEVICE;
    // the parameters (80 B each) are staged in the descriptor buffer (128 B each)
    aop_status st = ensure_stage(ctx, (size_t)n);
    if (st != AOP_OK) return st;
    aop::ApproxParam *prm = reinterpret_cast<aop::ApproxParam *>(ctx->h_stage);
    for (int64_t i = 0; i < n; ++i) {
        const aop_option &o = opts[i];
        aop::ApproxParam &q = prm[i];
        std::memset(&q, 0, sizeof(q));
        Desc d;
        aop_status s = make_desc(o, ctx->lambda, d);
        if (s == AOP_OK && o.model != AOP_BINOMIAL_CALL) s = AOP_ENOTIMPL;  // the section covers the binomial call
        if (h_status) h_status[i] = s;
        if (s != AOP_OK) continue;
        // Fig. 1: dt = E/T, u = e^{V sqrt(dt)}, p = (e^{(R-Y)dt} - 1/u)/(u - 1/u), m = e^{-R dt}
        const double T = (double)o.T, dt = o.expiry / T;
        const double a = o.sigma * std::sqrt(dt), u = std::exp(a), dn = 1.0 / u;
        const double p = (std::exp((o.r - o.q) * dt) - dn) / (u - dn);
        q.S = o.S0;
        q.K = o.K;
        q.a = a;
        q.mu = p * T;
        q.v = p * (1.0 - p) * T;
        q.disc = std::pow(std::exp(-o.r * dt), T);
        q.T = o.T;
        q.method = method;
        q.valid = 1;
        q.xlo = 0;
        q.xhi = o.T - 1;
        if (method == 0) {  // mean +- 6 standard deviations, clipped to [0, T-1]
            const double sd = std::sqrt(q.v);
            const double lo = std::ceil(q.mu - 6.0 * sd), hi = std::ceil(q.mu + 6.0 * sd);
            q.xlo = lo > 0.0 ? (int64_t)lo : 0;
            q.xhi = (hi < T ? (int64_t)hi : o.T) - 1;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(d_ws, prm, sizeof(aop::ApproxParam) * (size_t)n, hipMemcpyHostToDevice, s) != hipSuccess)
        return AOP_EDEVICE;
    if (hipEventRecord(ctx->stage_done, s) != hipSuccess) return AOP_EDEVICE;
    ctx->stage_pending = true;
    if (aop::launch_approx((const aop::ApproxParam *)d_ws, n, d_price, stream) != 0) return AOP_EDEVICE;
    return AOP_OK;
}

aop_status aop_plain_workspace_bytes(const aop_option *opts, int64_t n, size_t *bytes)
{
    if (!bytes || n < 0 || (n > 0 && !opts)) return AOP_EINVAL;
    std::vector<Desc> d((size_t)std::max<int64_t>(n, 1));
    *bytes = build_plain(opts, n, 1.0 / 3.0, d.data(), nullptr);
    return AOP_OK;
}

struct aop_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
};

aop_status aop_graph_create(aop_ctx *ctx, const aop_option *opts, int64_t n, int32_t precision, void *d_ws,
                            size_t ws_bytes, double *d_price, int32_t *h_status, int64_t *d_bnd,
                            int64_t bnd_stride, aop_graph **out)
{
    if (!ctx || !out || n <= 0 || !opts || !d_ws || !d_price) return AOP_EINVAL;
    *out = nullptr;
    if (hipSetDevice(ctx->device) != hipSuccess) return AOP_EDEVICE;
    std::vector<Desc> descs((size_t)n);
    std::vector<int32_t> stat((size_t)n);
    const size_t need = aop::build_batch(opts, n, precision, ctx->lambda, descs.data(), stat.data());
    if (h_status) std::memcpy(h_status, stat.data(), sizeof(int32_t) * (size_t)n);
    if (ws_bytes < need) return AOP_ENOMEM;
    if (d_bnd) {
        int64_t tmax = 0;
        for (int64_t i = 0; i < n; ++i) tmax = std::max<int64_t>(tmax, opts[i].T);
        if (bnd_stride < tmax + 1) return AOP_EINVAL;
    }
    // the descriptors are written once, outside the graph: a replay reads nothing from the host
    if (hipMemcpy(d_ws, descs.data(), sizeof(Desc) * (size_t)n, hipMemcpyHostToDevice) != hipSuccess)
        return AOP_EDEVICE;
    aop_graph *g = new (std::nothrow) aop_graph;
    if (!g) return AOP_ENOMEM;
    g->device = ctx->device;
    hipStream_t cs = nullptr;
    aop_status rc = AOP_OK;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) rc = AOP_EDEVICE;
    if (rc == AOP_OK && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = AOP_EDEVICE;
    if (rc == AOP_OK) {
        aop::Tune tune = aop::make_tune(*ctx, 0);
        tune.prec = precision;
        const int lr = aop::launch_solve((const Desc *)d_ws, n, (char *)d_ws, ctx->d_tw, d_price, d_bnd, bnd_stride,
                                         nullptr, tune, cs);
        const hipError_t e = hipStreamEndCapture(cs, &g->graph);
        if (lr != 0 || e != hipSuccess) rc = AOP_EDEVICE;
    }
    if (rc == AOP_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) rc = AOP_EDEVICE;
    if (cs) (void)hipStreamDestroy(cs);
    if (rc != AOP_OK) {
        aop_graph_destroy(g);
        return rc;
    }
    *out = g;
    return AOP_OK;
}

aop_status aop_graph_launch(aop_graph *g, void *stream)
{
    if (!g || !g->exec) return AOP_EINVAL;
    if (hipSetDevice(g->device) != hipSuccess) return AOP_EDEVICE;
    return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? AOP_OK : AOP_EDEVICE;
}

aop_status aop_graph_destroy(aop_graph *g)
{
    if (!g) return AOP_EINVAL;
    (void)hipSetDevice(g->device);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return AOP_OK;
}

aop_status aop_price_batch_plain(aop_ctx *ctx, const aop_option *opts, int64_t n, void *d_ws,
                                 size_t ws_bytes, double *d_price, int32_t *h_status, int64_t *d_bnd,
                                 int64_t bnd_stride, void *stream)
{
    if (!ctx || n < 0 || (n > 0 && (!opts || !d_ws || !d_price))) return AOP_EINVAL;
    if (n == 0) return AOP_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return AOP_EDEVICE;
    aop_status st = ensure_stage(ctx, (size_t)n);
    if (st != AOP_OK) return st;
    std::vector<int32_t> stat((size_t)n);
    const size_t need = build_plain(opts, n, ctx->lambda, ctx->h_stage, stat.data());
    if (h_status) std::memcpy(h_status, stat.data(), sizeof(int32_t) * (size_t)n);
    if (ws_bytes < need) return AOP_ENOMEM;
    if (d_bnd) {
        int64_t tmax = 0;
        for (int64_t i = 0; i < n; ++i) tmax = std::max<int64_t>(tmax, opts[i].T);
        if (bnd_stride < tmax + 1) return AOP_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(d_ws, ctx->h_stage, sizeof(Desc) * (size_t)n, hipMemcpyHostToDevice, s) != hipSuccess)
        return AOP_EDEVICE;
    if (aop::launch_plain_batch((const Desc *)d_ws, ctx->h_stage, n, (char *)d_ws, d_price, d_bnd, bnd_stride,
                                stream) != 0)
        return AOP_EDEVICE;
    if (hipEventRecord(ctx->stage_done, s) != hipSuccess) return AOP_EDEVICE;
    ctx->stage_pending = true;
    return AOP_OK;
}

aop_status aop_price(aop_ctx *ctx, const aop_option *opt, int32_t precision, double *h_price,
                     int64_t *h_bnd)
{
    if (!ctx || !opt || !h_price) return AOP_EINVAL;
    size_t bytes = 0;
    aop_status st = aop_workspace_bytes(opt, 1, precision, &bytes);
    if (st != AOP_OK) return st;
    int32_t ost = AOP_OK;
    {
        Desc d;
        ost = make_desc(*opt, ctx->lambda, d);
        if (ost == AOP_OK && precision != AOP_FP64 && precision != AOP_MIXED) ost = AOP_EINVAL;
        if (ost != AOP_OK) return (aop_status)ost;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return AOP_EDEVICE;
    void *ws = nullptr;
    double *dp = nullptr;
    int64_t *db = nullptr;
    const int64_t stride = opt->T + 1;
    aop_status rc = AOP_OK;
    if (hipMalloc(&ws, bytes) != hipSuccess || hipMalloc((void **)&dp, sizeof(double)) != hipSuccess ||
        (h_bnd && hipMalloc((void **)&db, sizeof(int64_t) * (size_t)stride) != hipSuccess)) {
        rc = AOP_ENOMEM;
    } else {
        rc = aop_price_batch(ctx, opt, 1, precision, ws, bytes, dp, &ost, db, stride, nullptr);
        if (rc == AOP_OK && hipStreamSynchronize(nullptr) != hipSuccess) rc = AOP_EDEVICE;
        if (rc == AOP_OK && hipMemcpy(h_price, dp, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
            rc = AOP_EDEVICE;
        if (rc == AOP_OK && h_bnd &&
            hipMemcpy(h_bnd, db, sizeof(int64_t) * (size_t)stride, hipMemcpyDeviceToHost) != hipSuccess)
            rc = AOP_EDEVICE;
        if (rc == AOP_OK && ost != AOP_OK) rc = (aop_status)ost;
    }
    if (ws) (void)hipFree(ws);
    if (dp) (void)hipFree(dp);
    if (db) (void)hipFree(db);
    return rc;
}

aop_status aop_batch_stats(const void *d_ws, int64_t n, aop_stats *h_stats)
{
    static_assert(sizeof(aop_stats) == sizeof(aop::Stats), "stats layout");
    if (!d_ws || !h_stats || n < 0) return AOP_EINVAL;
    if (n == 0) return AOP_OK;
    const char *src = (const char *)d_ws + aop::stats_offset(n);
    return hipMemcpy(h_stats, src, sizeof(aop_stats) * (size_t)n, hipMemcpyDeviceToHost) == hipSuccess
               ? AOP_OK
               : AOP_EDEVICE;
}

aop_status aop_batch_errors(const void *d_ws, int64_t n, int32_t *h_err)
{
    if (!d_ws || !h_err || n < 0) return AOP_EINVAL;
    if (n == 0) return AOP_OK;
    const char *src = (const char *)d_ws + aop::err_offset(n);
    return hipMemcpy(h_err, src, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost) == hipSuccess ? AOP_OK
                                                                                                  : AOP_EDEVICE;
}

aop_status aop_pool_stats(const void *d_ws, int64_t n, int64_t *h_out)
{
    if (!d_ws || !h_out || n < 0) return AOP_EINVAL;
    aop::PoolHdr hdr;
    if (hipMemcpy(&hdr, (const char *)d_ws + aop::pool_offset(n), sizeof(hdr), hipMemcpyDeviceToHost) != hipSuccess)
        return AOP_EDEVICE;
    h_out[0] = hdr.n_wg;
    h_out[1] = hdr.helper_tiles;
    h_out[2] = hdr.helper_busy;
    h_out[3] = hdr.helper_idle;
    h_out[4] = (int64_t)(hdr.status & 0xffffffffull);
    h_out[5] = (int64_t)(hdr.status >> 32);
    h_out[6] = 0;
    h_out[7] = 0;
    return AOP_OK;
}

aop_status aop_pool_abort_info(const void *d_ws, int64_t n, int64_t *h_out)
{
    if (!d_ws || !h_out || n < 0) return AOP_EINVAL;
    aop::PoolHdr hdr;
    if (hipMemcpy(&hdr, (const char *)d_ws + aop::pool_offset(n), sizeof(hdr), hipMemcpyDeviceToHost) != hipSuccess)
        return AOP_EDEVICE;
    for (int k = 0; k < 8; ++k) h_out[k] = hdr.abort_info[k];
    return AOP_OK;
}

aop_status aop_ctx_get_tuning(const aop_ctx *ctx, aop_tuning *out)
{
    if (!ctx || !out) return AOP_EINVAL;
    *out = ctx->tuning;
    return AOP_OK;
}

aop_status aop_ctx_set_tuning(aop_ctx *ctx, const aop_tuning *t)
{
    if (!ctx || !t) return AOP_EINVAL;
    aop_tuning u = *t;
    if (u.workgroups == 0) u.workgroups = std::min(ctx->n_cu, aop::MAX_WG);
    if (!aop::tuning_valid(u)) return AOP_EINVAL;
    ctx->tuning = u;
    return AOP_OK;
}

aop_status aop_sync(void *stream)
{
    return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? AOP_OK : AOP_EDEVICE;
}

}  // extern "C"
