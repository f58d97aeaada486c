// aop_host.h -- host-side internals shared by the C ABI (aop_api.cpp) and the
// serving engine (aop_serve.cpp); not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "aop.h"
#include "aop_internal.h"

struct aop_ctx {
    int device = 0;
    double lambda = 1.0 / 3.0;
    void *d_tw = nullptr;          // twiddle table, TW_N complex doubles (the caller's memory)
    aop::Desc *h_stage = nullptr;  // pinned staging for descriptors
    size_t stage_cap = 0;          // descriptors
    hipEvent_t stage_done = nullptr;
    bool stage_pending = false;
    int n_cu = 0;                  // compute units of the device
    double tick_hz = 1e8;          // device wall clock (s_memrealtime) frequency
    aop_tuning tuning{};           // launch tuning of the solve kernel
};

namespace aop {

constexpr size_t WS_ALIGN = 256;
inline size_t ws_align(size_t x) { return (x + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN; }

// Fill the descriptors of a batch (sorted by decreasing cost; out_index keeps
// the caller's order) and return the workspace bytes it needs.  status may be
// NULL.
size_t build_batch(const aop_option *opts, int64_t n, int32_t prec, double lambda, Desc *out, int32_t *status);

// Workspace bytes of one valid option's own area, and of a batch of n
// options without their areas (descriptors, counters, work pool).
size_t option_area_bytes(const aop_option &o, double lambda);
inline size_t batch_fixed_bytes(int64_t n) { return (size_t)options_offset(n); }

// Kernel tuning from public settings (device clock rate tick_hz), on
// `workgroups` workgroups (0: the settings' own).
Tune make_tune(const aop_tuning &t, double tick_hz, int32_t workgroups);
bool tuning_valid(const aop_tuning &t);
inline Tune make_tune(const aop_ctx &ctx, int32_t workgroups) { return make_tune(ctx.tuning, ctx.tick_hz, workgroups); }

}  // namespace aop
