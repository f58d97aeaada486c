/*
 * aop_cpu.h -- C ABI of libaop_cpu, the same FFT nonlinear-stencil method on
 * host cores with OpenMP tasks: the paper's own setting (Sec. 5 runs its
 * implementations on a 48-core machine with a base case of 8 time steps).
 * A comparison path beside the gfx950 library, never a fallback for it.
 *
 * Method: Sec. 2.3 ("Partitioning the triangle", "Solving a trapezoid") for
 * the binomial call, Sec. 3 for the trinomial call, Sec. 4.3 for the BSM put;
 * the two correlations of a trapezoid run as tasks beside its sub-trapezoids,
 * long FFTs split their butterfly stages into tasks, options run as tasks.
 */
#ifndef AOP_CPU_H
#define AOP_CPU_H

#include <stdint.h>

#include "aop.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Price n options (host memory throughout, synchronous).
 *   threads   OpenMP threads (0: the runtime's default).
 *   base      leaves of at most this many red cells are stepped directly
 *             (0: 8, the paper's best base case; 2..4096).
 *   lambda    dtau/ds^2 of the BSM grid (0: 1/3).
 *   price     n doubles (NaN where status != AOP_OK).
 *   status    NULL or n int32: the validation result of each option (the
 *             same rules as aop_validate).
 *   boundary  NULL or n * boundary_stride int64 (stride >= max T + 1): the
 *             per-row boundary with the meaning of aop_price_batch's.
 * Returns AOP_EINVAL for bad arguments, else AOP_OK.
 */
aop_status aop_cpu_price_batch(const aop_option *h_opts, int64_t n, int32_t threads, int32_t base,
                               double lambda, double *h_price, int32_t *h_status, int64_t *h_boundary,
                               int64_t boundary_stride);

#ifdef __cplusplus
}
#endif

#endif /* AOP_CPU_H */
