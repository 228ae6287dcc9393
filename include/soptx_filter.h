/* C ABI of the filter step of libsoptx (arXiv 2505.02438, Sec. 2.4 filtering
 * methods; Sec. 3.2 filter module: neighbourhoods searched once per mesh, the
 * filter held as a sparse matrix).
 *
 * The filter matrix H over the elements of a mesh:
 *     H_ij = max(0, r_min - dist(i, j)),
 * dist = Euclidean distance of the element centroids (the mean of the vertex
 * nodes: 4 for Q1 quads, 3 for P1 triangles, 8 for Q1 hexahedra, the 4
 * corners of P2 tetrahedra).  N_i = { j : H_ij > 0 } includes i (H_ii = r_min).
 * H is stored as CSR with int32 indices, columns ascending per row.
 *
 * Operations (all FP64, device pointers, n = number of elements):
 *   sensitivity filter   dc~_i  = sum_j H_ij rho_j dc_j / (max(1e-3, rho_i) sum_j H_ij)
 *   density filter       rho~_i = sum_j H_ij v_j rho_j / sum_j H_ij v_j   (v = element measure)
 *   Heaviside projection rho_bar_i = 1 - exp(-beta rho~_i) + rho~_i exp(-beta)
 *   their chain rule     dpsi/drho_j = v_j sum_i H_ij (dpsi/drho~_i) / (sum_k H_ik v_k),
 *                        dpsi/drho~_i = dpsi/drho_bar_i (beta exp(-beta rho~_i) + exp(-beta))
 * Each row is summed in ascending column order, each product rounded and
 * then added from zero: the order of a sequential CSR product (bitwise
 * reproducible, no atomics).
 *
 * Status codes are the SOPTX_* codes of soptx.h.  Device arrays must not
 * overlap between inputs and outputs of one call (SOPTX_E_INVALID_ARG when
 * an output equals an input).  Calls are asynchronous on `stream` (NULL =
 * default stream); calls on one stream are ordered.
 */
#ifndef SOPTX_FILTER_H
#define SOPTX_FILTER_H

#include <stdint.h>

#include "soptx.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct soptx_filter_s *soptx_filter;

/* Build H, the element measures v and the row sums sum_j H_ij v_j and
 * sum_j H_ij for a mesh (host memory, the checks of soptx_build_pattern_general:
 * SOPTX_E_BAD_MESH / _JACOBIAN / _NONAFFINE; Q1 cells may be non-affine, their
 * measure then the Gauss-rule integral of |det J|), by a uniform-cell neighbourhood
 * search, and copy them to the current device.  r_min > 0 and finite.
 * SOPTX_E_OVERFLOW when the number of stored entries exceeds int32.
 * Blocks until the uploads are complete.  *out receives a handle to release
 * with soptx_destroy_filter. */
int soptx_build_filter(const soptx_mesh *mesh, double rmin, soptx_filter *out, void *stream);

/* Flags of soptx_build_filter_ex. */
#define SOPTX_FILTER_CSR_ONLY 1 /* always apply H from its CSR form */

/* As soptx_build_filter.  Without SOPTX_FILTER_CSR_ONLY, H is also checked for
 * a stencil form: elements on a structured grid numbered lexicographically
 * (any axis order) and every row holding the same grid offsets with bitwise
 * equal weights (at most 512 offsets).  Then the products use the stencil and
 * read no H; the sums and results are the same as from the CSR form.
 * Unknown flag bits: SOPTX_E_INVALID_ARG. */
int soptx_build_filter_ex(const soptx_mesh *mesh, double rmin, int32_t flags, soptx_filter *out, void *stream);

/* Number of offsets of the stencil form of H, 0 when the CSR form is used. */
int soptx_filter_stencil_size(soptx_filter h, int32_t *S);

/* Number of elements and of stored entries of H; rows of H per thread block
 * of the product kernels (rows_per_block may be NULL). */
int soptx_filter_info(soptx_filter h, int64_t *n, int64_t *nnz, int32_t *rows_per_block);

/* Host copies of H (row_ptr [n+1], col [nnz], w [nnz]) and of the element
 * measures v [n]; any pointer may be NULL. */
int soptx_filter_copy(soptx_filter h, int32_t *h_row_ptr, int32_t *h_col, double *h_w, double *h_vol);

/* Sensitivity filter: d_dc_out[i] = dc~_i from d_rho [n] and d_dc [n]. */
int soptx_filter_sensitivity(soptx_filter h, const double *d_rho, const double *d_dc, double *d_dc_out,
                             void *stream);

/* Density filter: d_rho_tilde [n] = rho~ from the design d_rho [n].  With
 * d_rho_bar non-NULL also the Heaviside projection at beta (beta >= 0,
 * finite; beta = 0 gives rho_bar = rho~). */
int soptx_filter_density(soptx_filter h, const double *d_rho, double beta, double *d_rho_tilde,
                         double *d_rho_bar, void *stream);

/* Chain rule of the density filter: d_grad_rho [n] = dpsi/drho.  With
 * d_rho_tilde NULL, d_grad [n] holds dpsi/drho~; otherwise it holds
 * dpsi/drho_bar and is taken through the Heaviside projection at beta and
 * d_rho_tilde [n].  Uses a per-(device, stream) scratch vector of n doubles,
 * allocated on first use. */
int soptx_filter_density_backward(soptx_filter h, const double *d_rho_tilde, double beta, const double *d_grad,
                                  double *d_grad_rho, void *stream);

void soptx_destroy_filter(soptx_filter h);

#ifdef __cplusplus
}
#endif

#endif
