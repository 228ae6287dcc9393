/*
 * soptx_debug.h -- host-only introspection of the once-per-mesh build of
 * libsoptx (CSR pattern, element geometry and assembly plan), for tests and
 * tools.  None of these functions touches a device.
 *
 * The build is the one soptx_build_pattern performs before its uploads
 * (paper, Sec. 2.2: sparse K = sum_e E(rho_e) K_e^0; Sec. 3.2.2: invariant
 * components built once and reused).
 */
#ifndef SOPTX_DEBUG_H
#define SOPTX_DEBUG_H

#include <stdint.h>

#include "soptx.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct soptx_host_plan_s *soptx_host_plan;

/* Build pattern, geometry and plan on the host.  Same validation and error
 * codes as soptx_build_pattern.  *out is released with
 * soptx_debug_host_plan_free. */
int soptx_debug_host_plan(const soptx_mesh *mesh, soptx_host_plan *out);

/* As soptx_debug_host_plan; general != 0 builds the plan of
 * soptx_build_pattern_general (non-affine Q1 accepted, with the arrays gptr,
 * gent and gnode of the per-quadrature-point assembly). */
int soptx_debug_host_plan_ex(const soptx_mesh *mesh, int32_t general, soptx_host_plan *out);

/* Borrow one array of the plan by name: "row_ptr", "col_idx" (int32 CSR),
 * "geo" (double, [(dim*dim+1)][n_cells]: J^-1 row-major then det J),
 * "sig_info", "sig_pos_ptr", "sig_contrib", "sig_pairs", "sig_witems", "sig_witem_ptr", "grp_info", "grp_nodes",
 * "grp_elems", "grp_rows", "nb_tslot" (int32), "grp_n2l", "pos", "nb_tdeg" (uint16); for
 * general plans "gptr", "gent", "gnode" (int32) and, for Q1 elements, "qgeo"
 * (double, [NQ][dim][dim][n_cells]: sqrt(w_q |det J_q|) J_q^-1 at Gauss point
 * q per plan column, the element or, in a canonical-order plan, its rank).
 * The pointer stays valid until soptx_debug_host_plan_free. */
int soptx_debug_host_plan_array(soptx_host_plan p, const char *name, const void **data, int64_t *count,
                                int32_t *elem_bytes);

/* out8 = {ndof, nnz, n_groups, n_signatures, emax, kmax, dim, nen}. */
int soptx_debug_host_plan_scalars(soptx_host_plan p, int64_t *out8);

void soptx_debug_host_plan_free(soptx_host_plan p);

/* The filter matrix of soptx_build_filter (soptx_filter.h), built on the host
 * only (no device): sizes into *n and *nnz, and, for non-NULL buffers,
 * row_ptr [n+1], col [nnz], w [nnz], element measures vol [n] and the row
 * sums hsv [n] (sum_j H_ij v_j) and hs [n] (sum_j H_ij).  Call once with NULL
 * buffers to learn nnz. */
int soptx_debug_filter_matrix(const soptx_mesh *mesh, double rmin, int64_t *n, int64_t *nnz, int32_t *row_ptr,
                              int32_t *col, double *w, double *vol, double *hsv, double *hs);

/* Whether soptx_build_filter_ex would use the stencil form of H for this mesh
 * and radius (host only): *S = number of offsets (0: CSR form) and N [3] the
 * grid sizes, slowest axis first (zeros without a stencil). */
int soptx_debug_filter_stencil(const soptx_mesh *mesh, double rmin, int32_t *S, int64_t *N);

/* Test hook of the host build: the next n chunks of work that the pattern
 * and plan build hands to its worker threads fail as if an allocation had
 * failed, so that the build's error path (SOPTX_E_OOM, every thread joined)
 * can be exercised without exhausting memory.  n = 0 turns it off.
 * SOPTX_E_INVALID_ARG for n < 0. */
int soptx_debug_fail_workers(int32_t n);

/* Test hook: which assembly kernel the assembling calls launch, process-wide:
 * -1 = chosen from the plan (default: one workgroup per node group where a
 * group's stage is small or groups are few, the persistent warp-specialised
 * kernel otherwise), 0 = the persistent kernel, 1 = one workgroup per node
 * group.  All give bitwise the same K.  SOPTX_E_INVALID_ARG for other values. */
int soptx_debug_set_assembly_variant(int32_t v);

/* Test hook: how soptx_assemble_general assembles Q1 elements whose map is
 * not affine, process-wide.  The forms: (1) in LDS, one workgroup per node
 * group of the plan with the Jacobian at every Gauss point, the blocks'
 * sums in registers (plans with few work items per node group); (2) the
 * same with the sums in an LDS stage; (0) every element matrix written to
 * device memory, then one gather per block of K.  All sum each block's
 * contributions in ascending element order and differ in rounding only.
 * v = -1 (default): form 1 where the plan allows it, else 2 where its
 * largest group fits LDS, else 0; v = 0: form 0; v = 1: form 2 where it
 * fits, else 0.  Q2 hexahedra always take form 0.  SOPTX_E_INVALID_ARG for
 * other values. */
int soptx_debug_set_general_variant(int32_t v);

/* The form (1, 2 or 0 above) that soptx_assemble_general runs on handle h
 * (built by soptx_build_pattern_general) under the current variant, in
 * *form.  SOPTX_E_INVALID_ARG for a null argument or a handle without the
 * general tables. */
int soptx_debug_general_path(soptx_pattern h, int32_t *form);

#ifdef __cplusplus
}
#endif
#endif /* SOPTX_DEBUG_H */
