/*
 * aop.h -- C ABI of libaop, an MI355X (gfx950) library that prices American
 * options with the FFT-based nonlinear 1D stencil of Ahmad et al., "Fast
 * American Option Pricing using Nonlinear Stencils" (arXiv 2303.02317).
 *
 * Problem statement (Fig. 1, Table 1 notation): given spot S, strike K,
 * risk-free rate R, dividend yield Y, volatility V, time to expiry E and the
 * number of time steps T, return the option value at the root of
 *   - the binomial (CRR) lattice, American call          (Sec. 2, Def. 2.1),
 *   - the trinomial lattice, American call                (Sec. 3),
 *   - the explicit finite-difference BSM grid, American put (Sec. 4, eq. bsmG).
 * E is in years; dt = E/T.  The BSM grid uses s = ln(x/K), tau = sigma^2 t / 2,
 * dtau = sigma^2 E / (2T), ds = sqrt(dtau / lambda), centred on s0 = ln(S/K).
 *
 * The method (Sec. 2.3, Sec. 3, Sec. 4.3): a red (continuation) segment is
 * advanced many rows at once by correlating it with the h-step stencil kernel
 * through FFTs; the red/green boundary, which moves at most one cell per row
 * (Corollary 2.6, Theorem 4.2), is tracked by recursive trapezoid
 * decomposition whose base case is a narrow band of the direct
 * max(continuation, exercise) stencil.  Work O(T log^2 T), span O(T).
 *
 * Conventions
 *   - Pointers named d_* are device (HBM) pointers; h_* are host pointers.
 *   - Nothing here allocates device memory except the synchronous helper
 *     aop_price: the twiddle table, batch workspaces and the serving arena
 *     are the caller's (e.g. torch tensors).
 *   - All functions return an aop_status; nothing throws across the ABI.
 *   - A context is not thread-safe: use one context per host thread.
 *   - Ties between continuation and exercise value count as continuation
 *     (Def. 2.1: red when G^red >= G^green).  A cell whose exercise value is
 *     not finite is an exercise cell.
 */
#ifndef AOP_H
#define AOP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AOP_BINOMIAL_CALL = 0,  /* Sec. 2: CRR lattice, American call with dividend yield */
    AOP_TRINOMIAL_CALL = 1, /* Sec. 3: trinomial lattice, American call */
    AOP_BSM_PUT = 2         /* Sec. 4: explicit FD grid of the BSM PDE, American put (Y = 0) */
} aop_model;

typedef enum {
    AOP_FP64 = 0,  /* every step in IEEE double precision */
    AOP_MIXED = 1  /* FFT convolutions in FP32 split (hi/lo) arithmetic; boundary
                      search, band stencil and root accumulation in FP64 */
} aop_precision;

typedef enum {
    AOP_OK = 0,
    AOP_EINVAL = 1,    /* non-finite or non-positive S, K, V, E; T < 1; unknown model;
                          Y != 0 for the BSM put; bad lambda; unknown flag bits */
    AOP_EPROB = 2,     /* lattice probability outside (0,1), a BSM scheme
                          coefficient negative (explicit-scheme stability), or
                          an American trinomial call with R < 0 (outside the
                          hypotheses of the boundary lemmas of Sec. 3) */
    AOP_ENOMEM = 3,    /* workspace too small / allocation failed */
    AOP_EDEVICE = 4,   /* HIP runtime error */
    AOP_ETOOBIG = 5,   /* T above AOP_MAX_T */
    AOP_ECANCELED = 6, /* not priced: earlier failure in the same call */
    AOP_ENOTIMPL = 7   /* the requested precision is not available for this model */
} aop_status;

#define AOP_MAX_T (1LL << 21)

/* Option flags.  AOP_EUROPEAN: exercise at expiry only.  The method then
 * needs no boundary search: the root is one FFT correlation of the expiry
 * row (lattices: row T-1, computed directly from it) with the multi-step
 * stencil kernel, as in the paper's section on the European call under the
 * binomial model; boundary outputs hold -1 (lattices) or INT64_MIN (BSM)
 * below the expiry row, whose own entry is still reported. */
#define AOP_EUROPEAN 1

/* One option (host memory).  flags: 0 (American) or AOP_EUROPEAN.
 * exercise_every: 0 or 1 for the American (or, with AOP_EUROPEAN, European)
 * option; d >= 2 for a Bermudan binomial call, exercisable only on the rows i
 * with (T - i) % d == 0 -- every d time steps back from expiry (the paper's
 * closing section lists Bermudan options as future work; here the same
 * recursion steps from one exercise row to the next, so its cone widens by d
 * columns per step).  d > T leaves no exercise before expiry.  Only
 * AOP_BINOMIAL_CALL takes d >= 2 (others: AOP_ENOTIMPL); d >= 2 with
 * AOP_EUROPEAN is AOP_EINVAL. */
typedef struct {
    int32_t model;   /* aop_model */
    int32_t flags;
    double S0;       /* spot */
    double K;        /* strike */
    double r;        /* risk-free rate, continuously compounded, per year */
    double q;        /* dividend yield per year (must be 0 for AOP_BSM_PUT) */
    double sigma;    /* volatility per sqrt(year) */
    double expiry;   /* years */
    int64_t T;       /* time steps, 1 <= T <= AOP_MAX_T */
    int64_t exercise_every; /* 0/1 every row; d >= 2 Bermudan (binomial) */
} aop_option;

typedef struct aop_ctx aop_ctx;

/* Bytes of the FFT twiddle table a context needs (e^{-2 pi i t / 2^22},
 * t < 2^22, complex FP64: 64 MiB).  Used by the correlations of Sec. 2.3
 * ("Solving a trapezoid": each h-step kernel application is an FFT
 * correlation). */
size_t aop_twiddle_bytes(void);

/* Create a context on HIP device `device`.
 *   lambda      dtau/ds^2 of the BSM grid (Sec. 4.2, eq. bsmG; 0: the default
 *               1/3, at most 1/2 so that the scheme's coefficients stay >= 0).
 *   d_twiddles  device buffer of tw_bytes >= aop_twiddle_bytes(), 16-byte
 *               aligned, owned by the caller (e.g. a torch tensor); the context
 *               fills it (synchronously) and reads it until aop_ctx_destroy,
 *               which does not free it.
 * The context allocates no device memory; it holds a pinned host staging
 * buffer for descriptors.  Errors: AOP_EINVAL (bad lambda, NULL or misaligned
 * table), AOP_ENOMEM (table too small), AOP_EDEVICE. */
aop_status aop_ctx_create(int device, double lambda, void *d_twiddles, size_t tw_bytes, aop_ctx **out);
/* Release the context (not the caller's twiddle table). */
aop_status aop_ctx_destroy(aop_ctx *ctx);

/* Bytes of device workspace a batch of n options needs (host options): per
 * option two row buffers of the lattice (Fig. 1: row i of the binomial lattice
 * has i+1 cells; Sec. 3: 2i+1 trinomial cells; Sec. 4.2: the 2T+1-point BSM
 * cone), the recursion's middle rows (Sec. 2.3, "Solving a trapezoid") and
 * the FFT scratch, plus the batch's descriptors, counters and work pool.
 * Invalid options contribute nothing; their status is reported by the
 * pricing call. */
aop_status aop_workspace_bytes(const aop_option *h_opts, int64_t n, int32_t precision,
                               size_t *bytes);

/* Validate one option and report its status without pricing it: the
 * parameter checks of Fig. 1 (binomial p in (0,1)), Sec. 3 (trinomial
 * probabilities) and eq. bsmG (BSM coefficients >= 0); see aop_status. */
aop_status aop_validate(const aop_option *h_opt, double lambda);

/*
 * Price n options with the FFT nonlinear-stencil method (Sec. 2.3 for the
 * binomial call: "Partitioning the triangle" into trapezoids and "Solving a
 * trapezoid" recursively; Sec. 3 for the trinomial call; Sec. 4.3 for the BSM
 * put), asynchronously on `hip_stream` (a hipStream_t; NULL = default stream).
 * The price is the root value G[0][0] of Def. 2.1 (BSM: K v^T_0).
 *   h_opts      host array of n options (read before return).
 *   d_workspace device buffer of ws_bytes >= aop_workspace_bytes(); must stay
 *               alive and untouched until the stream reaches this work.
 *   d_price     device array of n doubles: the price of each option (NaN for
 *               an option whose status is not AOP_OK).
 *   h_status    host array of n int32 (written before return): AOP_OK or the
 *               validation error of each option.
 *   d_boundary  NULL, or a device array of n * boundary_stride int64 with
 *               boundary_stride >= max T + 1.  Row i (lattices) or step n (BSM)
 *               of option o goes to d_boundary[o * boundary_stride + i]:
 *               lattices: the last continuation column of row i, -1 if none;
 *               BSM: the last exercise offset k of step n, INT64_MIN if none.
 *               Rows the method never visits individually are exact too: every
 *               row is either walked by the band stencil or produced by it.
 * Returns AOP_OK when the batch was launched (per-option failures are in
 * h_status), AOP_ENOMEM if ws_bytes is too small, AOP_EDEVICE on HIP errors.
 */
aop_status aop_price_batch(aop_ctx *ctx, const aop_option *h_opts, int64_t n, int32_t precision,
                           void *d_workspace, size_t ws_bytes, double *d_price,
                           int32_t *h_status, int64_t *d_boundary, int64_t boundary_stride,
                           void *hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * pricing as aop_price_batch, with the workspace taken from a fixed array
 * inside the library, aop_noalloc_scratch_bytes() = 256 MiB per GPU, which
 * each GPU the library runs on holds until the process ends.  Allocates
 * nothing, host or device; the caller passes only the options and the output
 * buffers (d_price, h_status, d_boundary as in aop_price_batch).
 * Limits: n <= 256 options and a workspace (aop_workspace_bytes) of at most
 * 256 MiB -- e.g. one binomial option of T = 2^20, one trinomial option of
 * T = 2^19, or 64 options of T = 2^14; larger requests return AOP_ENOMEM
 * before anything is launched.  Every call on one GPU uses the same array and
 * leaves its contents behind: calls that overlap on one GPU (on different
 * streams, or from different contexts or threads) race and must be
 * serialised by the caller.  aop_batch_stats and friends do not apply.
 */
aop_status aop_price_batch_noalloc(aop_ctx *ctx, const aop_option *h_opts, int64_t n, int32_t precision,
                                   double *d_price, int32_t *h_status, int64_t *d_boundary,
                                   int64_t boundary_stride, void *hip_stream);
size_t aop_noalloc_scratch_bytes(void);

/*
 * Gaussian approximations of the European binomial call (the paper's section
 * on the European call under the binomial model): the up-move count of the
 * T-step lattice (Fig. 1) is replaced by a normal variable with mean pT and
 * variance p(1-p)T, and the price m^T E[(S u^{2x-T} - K)^+] is taken as
 *   method 0  the sum over integer x within 6 standard deviations of the
 *             mean (clipped to [0, T-1]): O(sqrt T) terms;
 *   method 1  the sum over x in [0, T-1]: O(T) terms;
 *   method 2  the integral over x from ceil(T/2 + ln(K/S)/(2 ln u)) to T in
 *             closed form with erf: O(1).
 * These are approximations of the lattice value (error of order 1/T for the
 * sums, larger for the integral), not the lattice value itself: the exact
 * European price is aop_price_batch with AOP_EUROPEAN.  Only
 * AOP_BINOMIAL_CALL is covered (others get status AOP_ENOTIMPL, price NaN);
 * exercise flags are ignored.  d_workspace: aop_approx_workspace_bytes(n)
 * device bytes (caller-owned); d_price: n doubles; h_status: n int32 (written
 * before return).  Asynchronous on hip_stream.
 */
size_t aop_approx_workspace_bytes(int64_t n);
aop_status aop_european_approx(aop_ctx *ctx, const aop_option *h_opts, int64_t n, int32_t method,
                               void *d_workspace, size_t ws_bytes, double *d_price, int32_t *h_status,
                               void *hip_stream);

/*
 * Graph form of aop_price_batch (same method and outputs; the launch form is
 * this library's, the paper runs on CPU cores): the batch's launch (clearing of the work
 * pool and the persistent solve kernel) is captured once in a hipGraph and
 * replayed with aop_graph_launch, for callers that price the same batch of
 * options repeatedly.  Arguments as in aop_price_batch (the graph uses the
 * context's tuning at creation time); the descriptors are written to
 * d_workspace synchronously during creation.  d_workspace, d_price and
 * d_boundary must stay allocated while the graph exists; each replay
 * overwrites d_price (and d_boundary) with the same prices.  Replays on one
 * workspace must not overlap.
 */
typedef struct aop_graph aop_graph;
aop_status aop_graph_create(aop_ctx *ctx, const aop_option *h_opts, int64_t n, int32_t precision,
                            void *d_workspace, size_t ws_bytes, double *d_price, int32_t *h_status,
                            int64_t *d_boundary, int64_t boundary_stride, aop_graph **out);
aop_status aop_graph_launch(aop_graph *graph, void *hip_stream);
aop_status aop_graph_destroy(aop_graph *graph);

/*
 * Comparison path: the plain Theta(T^2) backward induction of Fig. 1 (the
 * standard looping code; Table 2's Theta(T^2) work) on the GPU, every cell
 * updated with the direct max(continuation, exercise) stencil of Def. 2.1
 * (Sec. 3 trinomial, eq. bsmG for BSM).  Same arguments and semantics as
 * aop_price_batch, FP64 only (precision is not taken).  d_boundary: NULL or
 * n * boundary_stride int64 (boundary_stride >= max T + 1), the same
 * per-row boundary as aop_price_batch reports, found by scanning every cell.
 * Workspace: aop_plain_workspace_bytes (two row buffers per option).
 */
aop_status aop_plain_workspace_bytes(const aop_option *h_opts, int64_t n, size_t *bytes);
aop_status aop_price_batch_plain(aop_ctx *ctx, const aop_option *h_opts, int64_t n,
                                 void *d_workspace, size_t ws_bytes, double *d_price,
                                 int32_t *h_status, int64_t *d_boundary, int64_t boundary_stride,
                                 void *hip_stream);

/* Work an option's solve performed (written by the kernel into the workspace):
 * the correlations of Sec. 2.3 (two per trapezoid), the band rows of its base
 * case, and clock counters of where the driver spent its time. */
typedef struct {
    int64_t convs;        /* FFT correlations (h-step kernel applications) */
    int64_t conv_in;      /* sum of input lengths (doubles read from HBM) */
    int64_t conv_out;     /* sum of output lengths (doubles written to HBM) */
    int64_t fft_points;   /* sum of transform sizes N */
    int64_t band_rows;    /* row steps of the band stencil (the span) */
    int64_t direct_cells; /* cells of the expiry-adjacent row computed directly */
    int64_t max_depth;    /* deepest trapezoid recursion level */
    int64_t trapezoids;   /* top-level trapezoids */
    int64_t n_direct;     /* correlations evaluated by direct stepping */
    int64_t n_fft;        /* correlations evaluated by FFT */
    int64_t cyc_band;     /* driver's shader clock cycles in the band stencil */
    int64_t cyc_tiles;    /* ... computing correlation tiles itself */
    int64_t cyc_wait;     /* ... waiting for tiles other workgroups took */
    int64_t cyc_rows;     /* ... computing the rows next to expiry */
    int64_t cyc_total;    /* ... in the whole solve of the option */
    int64_t n_published;  /* correlations handed to the work pool */
} aop_stats;

/* Copy the work counters of the last aop_price_batch on this workspace to the
 * host (synchronous; call after the stream has passed the batch).  h_stats:
 * n entries in the caller's order; entries of rejected options are zero.
 * These counters give the algorithmic HBM bytes of the correlations (Sec. 2.3:
 * each reads its input segment and writes its output segment once). */
aop_status aop_batch_stats(const void *d_workspace, int64_t n, aop_stats *h_stats);

/* Device-side error code (this library's geometry and deadline checks, not a
 * quantity of the paper) of each option of the last aop_price_batch (or graph
 * replay) on this workspace, in the caller's order (synchronous): 0 none,
 * 1 a range check failed, 2 recursion stack, 3 arena or FFT scratch exhausted,
 * 5 a wait passed its deadline, 6 priced after the launch aborted.  An option
 * with a nonzero code has a NaN price. */
aop_status aop_batch_errors(const void *d_workspace, int64_t n, int32_t *h_err);

/* Work-pool counters (the pool runs the independent correlations of a
 * trapezoid, Sec. 2.3, on idle workgroups) of the last aop_price_batch on this workspace
 * (synchronous): h_out[0] workgroups, [1] tiles computed by helper
 * workgroups, [2] helper busy cycles, [3] helper idle cycles, [4] options
 * finished, [5] 1 if the launch aborted (a wait passed its deadline or a job was refused), [6..7] 0. */
aop_status aop_pool_stats(const void *d_workspace, int64_t n, int64_t h_out[8]);
/* Diagnostics of an aborted launch on this workspace (synchronous): h_out[0] the
 * first cause (0 none, 1 a helper refused a job's arguments, 2 a driver's wait
 * passed its deadline, 3 a wait while retiring jobs after an error passed its
 * deadline), h_out[1..6] details of that event (job slot, phase and tile or
 * control word, job kind and sizes, workgroup), h_out[7] 0. */
aop_status aop_pool_abort_info(const void *d_workspace, int64_t n, int64_t h_out[8]);

/*
 * Launch tuning of the FFT path (per context; changes no result, only speed).
 * The batch kernel is persistent: `workgroups` workgroups each drive one option
 * at a time (largest first) and, once no option is left, compute tiles of the
 * correlations other drivers publish (Sec. 2.3: the two correlations of a
 * trapezoid are independent of its sub-trapezoids).
 */
typedef struct {
    int32_t workgroups;     /* persistent grid (0 = one per compute unit, at most 512) */
    int32_t pub_min_lg;     /* FFT correlations of size >= 2^pub_min_lg are published (1..30) */
    int32_t pub_direct;     /* 1: publish direct-stepping correlations too; 0: run them inline */
    int32_t direct_max_h;   /* correlations with h <= this (<= 448, and n <= direct_max_n) step directly */
    int32_t direct_max_n;   /* <= 2048 */
    int32_t helper_idle_us; /* a helper workgroup leaves after this long without work (>= 1) */
    int32_t late_pub_min_lg; /* once late_after_pct % of the launch's options are done, the drivers
                                still running publish FFT correlations of size >= 2^this (0 = never) */
    int32_t late_after_pct;  /* 0..100 */
    int32_t lds_max_lg;     /* FP64 correlations of up to 2^this points run as one LDS transform,
                               longer ones as four-step transforms of 2048-point rows (11 or 12) */
    int32_t radix_lg;       /* FP64 LDS butterfly passes of radix 2^radix_lg (2 or 3) */
    int64_t timeout_ms;     /* a wait longer than this aborts the launch: its options price NaN (> 0) */
    int64_t timeout_us;     /* > 0: the same deadline in microseconds, in place of timeout_ms (callers that
                               need one below a millisecond); 0: timeout_ms applies */
} aop_tuning;
aop_status aop_ctx_get_tuning(const aop_ctx *ctx, aop_tuning *out);
/* Returns AOP_EINVAL (and keeps the old tuning) for out-of-range fields. */
aop_status aop_ctx_set_tuning(aop_ctx *ctx, const aop_tuning *tuning);

/*
 * Serving: continuous batching of pricing requests of mixed model and T,
 * priced by the persistent FFT-path kernel while new requests keep arriving.
 *
 * (The paper prices one option at a time; serving is this library's form of
 * the same method for request streams: each request is priced exactly as by
 * aop_price_batch, Sec. 2.3 / 3 / 4.3.)
 *
 * A server uses a device arena of hbm_budget bytes that the caller owns (its
 * HBM budget) and a
 * scheduler thread with max_inflight launch slots, each with its own HIP
 * stream and 1/max_inflight of the compute units.  When a slot is free the
 * scheduler takes the oldest pending request, adds younger requests of the same
 * size class (model, ceil(log2 T)) in arrival order up to max_batch while the
 * batch's workspace still fits in one free block of the arena (admission by
 * HBM footprint), and launches it; batches admitted while others run overlap
 * on the device.  Each option's schedule depends only on that option, so its
 * price is bitwise the same alone and in any mix.
 *
 * The server uses the context's twiddle table and tuning: do not change the
 * context's tuning, nor destroy it, while a server on it exists.  The server
 * functions are thread-safe among themselves (submit and poll may run on
 * different threads).
 */
typedef struct aop_server aop_server;

/* Tuning of one size class (the autotuner's output); workgroups is ignored by
 * the server, which gives each batch 1/max_inflight of the compute units. */
typedef struct {
    int32_t model;      /* aop_model */
    int32_t log2T;      /* ceil(log2 T) of the class */
    int32_t precision;  /* aop_precision */
    int32_t reserved;   /* must be 0 */
    aop_tuning tuning;
} aop_class_tuning;

typedef struct {
    size_t hbm_budget;    /* bytes of d_arena the server may use for workspaces */
    int32_t max_inflight; /* batches on the device at once, 1..16 */
    int32_t max_batch;    /* options per batch, 1..4096 */
    int32_t precision;    /* AOP_FP64 or AOP_MIXED, for every request */
    int32_t reserved;     /* must be 0 */
    const aop_class_tuning *tunings; /* NULL, or n_tunings per-class schedules (copied at creation):
                                        a batch uses the entry of its model and precision nearest
                                        in log2T, else the context's tuning */
    int64_t n_tunings;
    void *d_arena;        /* device buffer of hbm_budget bytes, 256-byte aligned, owned by the
                             caller (e.g. a torch tensor); must outlive the server */
} aop_server_config;

typedef struct {
    uint64_t id;         /* the caller's request id */
    double price;        /* NaN unless status == AOP_OK */
    int32_t status;      /* AOP_OK, the option's validation error, AOP_ENOMEM (larger than the whole
                            budget), AOP_EDEVICE, or AOP_ECANCELED (server stopped on an error) */
    int32_t batch_size;  /* options in the launch that priced it (0 if none) */
    double queue_s;      /* seconds from submission to its launch */
    double latency_s;    /* seconds from submission to the result being available on the host */
} aop_result;

/* Start a server on the caller's arena (allocates no device memory: streams,
 * events and pinned host buffers only).  AOP_EINVAL for a bad configuration or
 * a NULL / misaligned arena. */
aop_status aop_server_create(aop_ctx *ctx, const aop_server_config *cfg, aop_server **out);
/* Queue n requests (host arrays, copied before return); arrival time is now. */
aop_status aop_server_submit(aop_server *server, const aop_option *h_opts, const uint64_t *h_ids, int64_t n);
/* Move up to max finished results to h_out (any order), waiting up to wait_us
 * microseconds for the first one; *n_out = number written.  Returns the
 * server's error state (AOP_OK while healthy). */
aop_status aop_server_poll(aop_server *server, aop_result *h_out, int64_t max, int64_t *n_out, int32_t wait_us);
/* h_out[0] submitted, [1] completed, [2] batches launched, [3] batches in flight,
 * [4] requests pending, [5] peak arena bytes in use, [6] arena bytes, [7] workgroups per batch,
 * [8] algorithmic HBM bytes of the finished batches (8 bytes per correlation input and output
 * cell and per directly computed cell, as aop_stats counts them). */
aop_status aop_server_stats(aop_server *server, int64_t h_out[9]);
/* Finish every queued request, then release the server's device memory and streams. */
aop_status aop_server_destroy(aop_server *server);

/* Synchronous convenience: price one option as aop_price_batch does (Sec. 2.3
 * / 3 / 4.3), allocating and freeing its own device workspace -- the one entry
 * point that allocates device memory.  h_boundary: NULL or a host array of
 * T+1 int64. */
aop_status aop_price(aop_ctx *ctx, const aop_option *h_opt, int32_t precision, double *h_price,
                     int64_t *h_boundary);

/* Wait for all work on hip_stream (plumbing, no quantity of the paper). */
aop_status aop_sync(void *hip_stream);

/* Text of a status code (plumbing). */
const char *aop_status_str(aop_status s);

/* Library version string. */
const char *aop_version(void);

#ifdef __cplusplus
}
#endif

#endif /* AOP_H */
