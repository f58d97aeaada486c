// aop_internal.h -- descriptor layout shared by the host API and the gfx950
// kernels of libaop (not part of the public ABI).
#pragma once
#include <stdint.h>

namespace aop {

enum Model : int32_t { BINOMIAL = 0, TRINOMIAL = 1, BSM = 2 };

// Sentinel of "no exercise cell" for the BSM boundary output.
constexpr int64_t BSM_NONE = INT64_MIN;

// Error codes an option's kernel can record (in Desc::dev_err) when one of
// its internal geometry checks fails; the option's price is then NaN.
enum DevErr : int32_t { DEV_OK = 0, DEV_RANGE = 1, DEV_STACK = 2, DEV_ARENA = 3, DEV_FFT = 4, DEV_TIMEOUT = 5, DEV_ABORT = 6 };

// Per-option descriptor, built on the host from the paper's formulas and
// copied to the device (128 bytes).
struct Desc {
    int32_t model;   // Model
    int32_t prec;    // 0 FP64, 1 mixed
    int64_t T;       // time steps
    double S, K;     // spot, strike
    double a;        // exercise exponent step: binomial a = V sqrt(dt) (S e^{(2j-i)a}),
                     // trinomial A = V sqrt(2 dt) (S e^{(j-i)A}), BSM ds (1 - e^{s0 + k ds})
    double s0;       // BSM: ln(S/K); 0 otherwise
    double w0, w1, w2;  // one-step stencil: binomial (w_dn on j, w_up on j+1, 0);
                        // trinomial (m p_d on j, m p_o on j+1, m p_u on j+2);
                        // BSM (b on k-1, c on k, a on k+1)
    int64_t ws_off;     // byte offset of this option's area in the workspace
    int64_t row_len;    // doubles per row buffer
    int64_t arena_len;  // doubles in the recursion arena
    int64_t nfft;       // complex elements in the FFT scratch
    int64_t out_index;  // index of this option in the caller's arrays
    int32_t no_green;   // lattice call with Y = 0, R >= 0: no exercise cell below the expiry row (Lemma 2.3)
    int32_t ex_every;   // exercise rows: 1 every row (American), 0 none before expiry (European),
                        // d >= 2 the rows i with (T - i) % d == 0 (Bermudan, binomial call only)
    int64_t scr_len;    // complex elements of FFT scratch (a stack shared by the outstanding correlations)
};
static_assert(sizeof(Desc) == 128, "descriptor is 128 bytes");

// Whether row i (lattices; step T - i) of an option may exercise.
#if defined(__HIPCC__)
__host__ __device__
#endif
inline bool exercise_row(const Desc &d, int64_t i)
{
    return d.ex_every == 1 || (d.ex_every > 1 && (d.T - i) % d.ex_every == 0);
}

// Per-option work counters (mirror of aop_stats), stored after the descriptors.
struct Stats {
    int64_t convs, conv_in, conv_out, fft_points, band_rows, direct_cells, max_depth, trapezoids;
    int64_t n_direct, n_fft, cyc_band, cyc_tiles, cyc_wait, cyc_rows, cyc_total, n_published;
};
static_assert(sizeof(Stats) == 128, "stats are 128 bytes");
inline int64_t stats_offset(int64_t n) { return ((int64_t)sizeof(Desc) * (n > 0 ? n : 1) + 255) / 256 * 256; }

// Work pool of the persistent solve kernel, after the stats region: a
// 128-byte header, a summary bitmap (bit w: workgroup w has a job slot with
// claimable tiles), one 64-bit word per workgroup whose bits flag those slots,
// and JPW job slots per workgroup (128 B each).
constexpr int JPW = 64;          // job slots per workgroup
constexpr int MAX_WG = 512;      // largest persistent grid
struct PoolHdr {
    uint32_t next_option, n_wg;
    uint64_t status;  // options finished (low 32 bits) | launch aborted (bit 32)
    int64_t helper_tiles, helper_busy, helper_idle;
    int64_t abort_info[8];  // first cause of an abort: reason (1 refused job, 2 wait deadline, 3 drain deadline), details
    int64_t n_helpers;  // workgroups that have entered the helper loop (arrival rank: home option)
    int64_t reserved[2];
};
static_assert(sizeof(PoolHdr) == 128, "pool header is 128 bytes");
constexpr int64_t JOB_BYTES = 128;
constexpr int64_t POOL_SUMMARY = 128;                 // byte offset of the summary bitmap (up to 1024 bits)
constexpr int64_t POOL_BITS = 256;                    // byte offset of the per-workgroup slot words
constexpr int64_t POOL_JOBS = POOL_BITS + 8 * MAX_WG; // byte offset of the job slots
constexpr int64_t POOL_DRV = POOL_JOBS + JOB_BYTES * JPW * MAX_WG;  // int32 per option (first MAX_WG): its driver
constexpr int64_t POOL_BYTES = POOL_DRV + 4 * MAX_WG;
// Per-option device error codes (DevErr, int32) after the counters.
inline int64_t err_offset(int64_t n)
{
    return stats_offset(n) + ((int64_t)128 * (n > 0 ? n : 1) + 255) / 256 * 256;
}
inline int64_t pool_offset(int64_t n) { return err_offset(n) + ((int64_t)4 * (n > 0 ? n : 1) + 255) / 256 * 256; }
inline int64_t options_offset(int64_t n) { return pool_offset(n) + POOL_BYTES; }

// Launch-time tuning of the solve kernel (device clock units).
struct Tune {
    int32_t workgroups;    // persistent grid size
    int32_t pub_min_lg;    // FFT correlations of size >= 2^pub_min_lg go to the pool
    int32_t pub_direct;    // direct-stepping correlations go to the pool (1) or run inline (0)
    int32_t direct_max_h;  // longest kernel evaluated by direct stepping
    int32_t direct_max_n;  // longest segment evaluated by direct stepping (<= 1024)
    int32_t prec;          // precision of the batch (every descriptor's): 0 FP64, 1 split-FP32 FFT
    int32_t late_pub_lg;   // publication threshold once late_after options are done (0: never)
    int32_t late_after;    // options done (set per launch from the percentage)
    int32_t lds_lg64;      // FP64 transforms of up to 2^lds_lg64 points run whole in LDS (11 or 12)
    int32_t radix;         // FP64 LDS butterfly passes of radix 2^radix (2 or 3)
    int64_t timeout_ticks; // wall-clock ticks a wait may take before the launch aborts
    int64_t idle_ticks;    // wall-clock ticks a helper waits for work before it leaves
};

// Spectrum cache of a driver: SPC_E kernel spectra of correlations of up to
// 2^SPC_LG points (bins 0 .. N/2), after the option's FFT scratch.
constexpr int SPC_LG = 12;
constexpr int SPC_E = 32;
constexpr int64_t spc_entry(int64_t nfft)  // complex elements per cache entry
{
    const int64_t n = nfft < (int64_t(1) << SPC_LG) ? nfft : (int64_t(1) << SPC_LG);
    return (n / 2 + 1 + 15) / 16 * 16;
}
constexpr int DIRECT_MAX_N = 2048;  // longest directly stepped correlation (in segments of <= 1024 cells)
constexpr int DIRECT_MAX_H = 448;   // deepest directly stepped correlation (its halo leaves room in a segment)
constexpr int LG_TW = 22;  // twiddle table: e^{-2 pi i t / 2^22}, t < 2^22
constexpr int64_t TW_N = int64_t(1) << LG_TW;

// Parameters of one Gaussian approximation of a European binomial call
// (80 bytes; built on the host from Fig. 1's lattice parameters).
struct ApproxParam {
    double S, K;      // spot, strike
    double a;         // ln u = V sqrt(dt)
    double mu, v;     // mean pT and variance p(1-p)T of the up-move count
    double disc;      // m^T
    int64_t T;
    int32_t method;   // 0 window of 6 sd, 1 sum over [0, T-1], 2 erf closed form
    int32_t valid;    // 0: rejected on the host (price NaN)
    int64_t xlo, xhi; // summation range (methods 0 and 1)
};
static_assert(sizeof(ApproxParam) == 80, "approximation parameters are 80 bytes");

// Host-side launchers (defined in aop_solver.hip / aop_plain.hip / aop_approx.hip).
int launch_twiddles(void *d_tw, void *stream);
int launch_solve(const Desc *d_desc, int64_t n, char *d_ws, const void *d_tw, double *d_price,
                 int64_t *d_bnd, int64_t bnd_stride, int32_t *d_err, const Tune &tune, void *stream);
int launch_approx(const ApproxParam *d_prm, int64_t n, double *d_price, void *stream);
int launch_plain_batch(const Desc *d_desc, const Desc *h_desc, int64_t n, char *d_ws, double *d_price,
                       int64_t *d_bnd, int64_t bnd_stride, void *stream);

}  // namespace aop
