/* C ABI of the optimality-criteria (OC) update of libsoptx (arXiv
 * 2505.02438, Sec. 2.3: the update factor B_e, the heuristic update with move
 * limit and damping, and Algorithm 1's bisection on the multiplier lambda).
 *
 * For design variables rho, objective sensitivities dc and volume-constraint
 * sensitivities dv (all with respect to the design variables; dv > 0):
 *     B_e(lambda)      = max(0, -dc_e) / (lambda dv_e)
 *     rho_new_e(lambda) = rho_e B_e^eta clamped to [max(0, rho_e - m), min(1, rho_e + m)]
 *     vol(lambda)      = sum_e dv_e rho_new_e(lambda)
 * (compliance sensitivities are <= 0; a positive dc_e is read as B_e = 0).
 * lambda is found by bisection: l1 = 0, l2 = lmax; while l2 - l1 > tol (l1 + l2)
 * and fewer than max_steps steps: mid = (l1 + l2) / 2, l1 = mid if
 * vol(mid) > vol_target else l2 = mid.  The result is rho_new at the last mid.
 * With dv the plain element measures, vol is the material volume; with dv
 * taken through the density filter's chain rule, vol equals the volume of the
 * filtered density exactly (the filter is linear in rho).
 *
 * The kernels take the same decisions as the sequential loop: each pass
 * evaluates the 15 midpoints the next 4 steps can visit (computed as the loop
 * computes them) and one block walks them.  vol is summed in a fixed order.
 *
 * Status codes are the SOPTX_* codes of soptx.h.
 */
#ifndef SOPTX_OC_H
#define SOPTX_OC_H

#include <stdint.h>

#include "soptx.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double move;       /* move limit m, 0 < m <= 1 */
    double eta;        /* damping exponent, 0 < eta <= 1 (0.5: square root) */
    double lmax;       /* initial upper end of the bracket, finite, > 0 */
    double tol;        /* relative width that ends the bisection, 0 < tol < 1 */
    int32_t max_steps; /* cap on bisection steps, 1 .. 1000 */
} soptx_oc_params;

typedef struct {
    double lambda; /* the last midpoint (the multiplier used for rho_new) */
    double volume; /* vol(lambda) */
    double change; /* max_e |rho_new_e - rho_e| */
    int32_t steps; /* bisection steps taken */
} soptx_oc_result;

/* One OC update of n design variables (device arrays of n doubles on the
 * current device; d_rho_new must not overlap the inputs).  Runs on `stream`
 * (NULL = default) and blocks
 * until the result is on the host (*out).  n = 0: nothing runs, *out is zero.
 * Uses a per-(device, stream) scratch, allocated on first use.
 * SOPTX_E_INVALID_ARG for a null pointer, n < 0, vol_target not finite or a
 * parameter out of range. */
int soptx_oc_update(int64_t n, const double *d_rho, const double *d_dc, const double *d_dv, double vol_target,
                    const soptx_oc_params *params, double *d_rho_new, soptx_oc_result *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif
