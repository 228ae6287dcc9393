/*
 * soptx.h -- C ABI of the MI355X (gfx950) SIMP assembly / compliance /
 * sensitivity library (libsoptx.so).
 *
 * The operations follow arXiv 2505.02438 (SOPTX):
 *   - modified SIMP law E(rho) = Emin + rho^p (E0 - Emin)       (Sec. 2.1)
 *   - K(rho) = sum_e E(rho_e) K_e^0, K_e^0 at unit modulus       (Sec. 2.2, Eq. cmpd)
 *   - c = F^T U = U^T K U, twice the strain energy               (Sec. 2.2, Eq. cmpc/cmpd)
 *   - dc/drho_e = -p rho_e^(p-1) (E0 - Emin) u_e^T K_e^0 u_e     (Appendix D)
 *   - "fast assembly": K_e^0 built from an element-independent reference
 *     tensor and element-dependent geometry (Sec. 3.2.2 solver module,
 *     Sec. 5.5); "symbolic" variant integrates the reference tensor exactly.
 *   - linear elastic isotropic material, plane stress in 2D by default
 *     (Sec. 3.2.1, Sec. 4.2).
 *
 * Conventions
 *   - Degrees of freedom are interleaved: dof = dim * node + component.
 *   - Element local node orders:
 *       SOPTX_QUAD4  (0,0),(1,0),(1,1),(0,1) counter-clockwise;
 *       SOPTX_TRI3   counter-clockwise vertices;
 *       SOPTX_HEX8   bottom face counter-clockwise, then top face;
 *       SOPTX_TET10  4 positively oriented vertices, then the nodes of
 *                    edges 01,02,03,12,13,23;
 *       SOPTX_HEX27  27-node triquadratic Lagrange hexahedron: the 8 corners
 *                    as for SOPTX_HEX8, then the other 19 points of the
 *                    reference lattice {0, 1/2, 1}^3, (a, b, c) / 2 with
 *                    a, b, c in {0, 1, 2}, in ascending a + 3b + 9c.
 *     Elements must be affine (parallelogram / parallelepiped Q1 cells,
 *     straight-edged P2 cells); others are rejected with SOPTX_E_NONAFFINE,
 *     except by the per-quadrature-point calls (soptx_*_general), which take
 *     general Q1 cells and SOPTX_HEX27, the latter only there.  SOPTX_HEX27
 *     is a higher-order variant beyond the paper's examples, which use linear
 *     elements (Sec. 3.2.2); the paper's platform offers any order (Sec. 1).
 *   - CSR pattern: the set {(dof(e,i), dof(e,j))}; rows ascending, columns
 *     ascending and unique per row; structural zeros are kept.  int32 indices.
 *   - Summation order of every stored K value is fixed by the mesh (the
 *     assembly plan built once per mesh), independent of the stream, of other
 *     work on the device and of the run: results are bitwise reproducible.
 *
 * Memory ownership
 *   - Host arrays passed to soptx_build_pattern are read during the call only.
 *   - The pattern handle owns every device copy it makes (pattern, plan,
 *     geometry, reference tensor) until soptx_destroy_pattern.
 *   - All per-call arrays named d_* are device pointers owned by the caller;
 *     they must stay valid until the stream reaches the call.
 *   - A handle is immutable after it is built: concurrent calls on different
 *     streams with the same handle are safe.  Destroy it only after every
 *     stream that used it has completed.
 *
 * Errors
 *   - Every int-returning function returns SOPTX_OK (0) or a negative code.
 *   - Argument and mesh validation happens before any device work, so on a
 *     validation error no output is touched.
 *   - Kernel launch failures are reported as SOPTX_E_DEVICE; faults inside
 *     kernels surface at the next synchronisation of that stream.
 *   - No exception or abort crosses this interface.
 *   - Per-call functions are asynchronous with respect to the host on
 *     `stream` (a hipStream_t; NULL = the default stream).
 */
#ifndef SOPTX_H
#define SOPTX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SOPTX_OK 0
#define SOPTX_E_INVALID_ARG (-1)      /* null pointer, bad size or enum */
#define SOPTX_E_UNSUPPORTED_ELEM (-2) /* element type not one of soptx_elem, or not taken by this call */
#define SOPTX_E_BAD_MESH (-3)         /* node index out of range, node repeated in a cell */
#define SOPTX_E_JACOBIAN (-4)         /* element with det J <= 0 (inverted or degenerate) */
#define SOPTX_E_NONAFFINE (-5)        /* element map is not affine */
#define SOPTX_E_OVERFLOW (-6)         /* nnz, dof count or a plan index exceeds its int32 range */
#define SOPTX_E_OOM (-7)              /* device or host allocation failed */
#define SOPTX_E_DEVICE (-8)           /* HIP runtime / launch error */
#define SOPTX_E_SCRATCH (-9)          /* input exceeds the fixed scratch of an allocation-free call */

typedef enum { SOPTX_QUAD4 = 1, SOPTX_TRI3 = 2, SOPTX_HEX8 = 3, SOPTX_TET10 = 4, SOPTX_HEX27 = 5 } soptx_elem;

/* Precision of the element-matrix contraction and of the element energy.
 * K values, the compliance and the cross-element accumulation are FP64 in
 * every form.  rho / dc / drho arrays are double for SOPTX_FP64 and float for
 * SOPTX_FP32.  SOPTX_BF16_FP32ACC (bf16 inputs, FP32 accumulation) is refused
 * by every call with SOPTX_E_INVALID_ARG: with bf16 operands the assembled K
 * is off by 4e-3 to 9e-3 (row-scaled) against the FP64 result, far outside
 * the 1e-5 bound that the FP32 form holds, so the form is not offered. */
typedef enum { SOPTX_FP64 = 0, SOPTX_FP32 = 1, SOPTX_BF16_FP32ACC = 2 } soptx_precision;

/* How the element-independent reference tensor is integrated (Sec. 5.5):
 * exactly in rational arithmetic ("symbolic fast assembly") or by the
 * element's exact quadrature rule in FP64 ("fast assembly"). */
typedef enum { SOPTX_REF_SYMBOLIC = 0, SOPTX_REF_QUADRATURE = 1 } soptx_ref_method;

/* Mesh (host memory).  coords: [n_nodes][dim] doubles; cells: [n_cells][nen]
 * node ids in the local order above.  dim must match elem. */
typedef struct {
    int32_t elem;
    int32_t dim;
    int64_t n_nodes;
    const double *coords;
    int64_t n_cells;
    const int32_t *cells;
} soptx_mesh;

/* Material (Sec. 3.2.1, Sec. 4.2): solid modulus E0, void modulus Emin
 * (Emin = 1e-9 E0 in the paper), Poisson ratio nu, SIMP exponent p.
 * plane_strain = 0 selects plane stress in 2D; ignored in 3D.
 * Requires E0 > Emin > 0, -1 < nu < 0.5, p >= 1. */
typedef struct {
    double E0, Emin, nu, p;
    int32_t plane_strain;
} soptx_material;

typedef struct soptx_pattern_s *soptx_pattern;

/* Statistics of a built pattern and its assembly plan. */
typedef struct {
    int64_t ndof, nnz, n_cells, n_nodes;
    int64_t n_groups;        /* node groups of the assembly plan */
    int64_t n_signatures;    /* distinct local-connectivity signatures */
    int64_t n_contributions; /* sum over elements of nen^2 block contributions */
    int64_t plan_bytes;      /* device bytes of the assembly plan (beyond the CSR pattern) */
    int64_t device_bytes;    /* all device bytes held by the handle */
    int64_t n_groups_diag;   /* groups whose elements all have a diagonal J^-1 (axis-aligned boxes),
                                assembled with the shorter contraction of such elements */
    int64_t n_groups_ranked; /* groups that carry a rank table: the plan took the canonical order of
                                nodes and elements (the given numbering fragmented it) */
} soptx_pattern_stats;

/* Build the CSR pattern, the per-element geometry (J^-1, det J) and the
 * assembly plan of a mesh, and copy them to the current device
 * (Sec. 2.2 sparse K; Sec. 3.2.2 "avoid recomputing invariant components").
 * Runs once per mesh; blocks until the device copies are complete.
 * On success *out receives a handle to release with soptx_destroy_pattern.
 * stream: used for the uploads (NULL = default stream). */
int soptx_build_pattern(const soptx_mesh *mesh, soptx_pattern *out, void *stream);

/* As soptx_build_pattern, choosing how the reference tensor is integrated. */
int soptx_build_pattern_ex(const soptx_mesh *mesh, int32_t ref_method, soptx_pattern *out,
                           void *stream);

/* Pattern sizes and its device arrays (owned by h, valid until destroy):
 * d_row_ptr: [ndof+1] int32; d_col_idx: [nnz] int32.  Any output may be NULL. */
int soptx_pattern_info(soptx_pattern h, int64_t *ndof, int64_t *nnz, const int32_t **d_row_ptr,
                       const int32_t **d_col_idx);

int soptx_pattern_stats_get(soptx_pattern h, soptx_pattern_stats *out);

/* Copy the device pattern to host arrays (h_row_ptr: [ndof+1], h_col_idx:
 * [nnz]; either may be NULL).  Blocks until the copies are done. */
int soptx_pattern_copy(soptx_pattern h, int32_t *h_row_ptr, int32_t *h_col_idx);

/* K_vals[slot(r,c)] = sum_e E(rho_e) K_e^0[r,c]  (Eq. cmpd), FP64.
 * d_rho: [n_cells] (double for SOPTX_FP64, float otherwise).
 * d_dirichlet: NULL, or [ndof] uint8 with nonzero = fixed dof; then every
 *   fixed dof r gets K[r,:] = 0, K[:,r] = 0, K[r,r] = 1 (zero prescribed
 *   values, Appendices A-C); the pattern is unchanged.
 * d_K_vals: [nnz] double, fully overwritten.
 * prec: SOPTX_FP64 or SOPTX_FP32 (SOPTX_E_INVALID_ARG otherwise). */
int soptx_assemble(soptx_pattern h, const soptx_material *m, const void *d_rho,
                   const uint8_t *d_dirichlet, double *d_K_vals, int32_t prec, void *stream);

/* The Dirichlet step of soptx_assemble on its own: for every fixed dof r of
 * d_dirichlet ([ndof] uint8, nonzero = fixed), K[r,:] = 0, K[:,r] = 0,
 * K[r,r] = 1 in d_K_vals ([nnz] double, the other entries untouched).
 * soptx_assemble with a mask equals soptx_assemble without one followed by
 * this call (zero prescribed values, Appendices A-C). */
int soptx_apply_dirichlet(soptx_pattern h, const uint8_t *d_dirichlet, double *d_K_vals, void *stream);

/* dc_e = -p rho_e^(p-1) (E0-Emin) u_e^T K_e^0 u_e  (Appendix D).
 * d_u: [ndof] double; d_dc: [n_cells] (double for SOPTX_FP64, float otherwise). */
int soptx_sensitivity(soptx_pattern h, const soptx_material *m, const void *d_rho,
                      const double *d_u, void *d_dc, int32_t prec, void *stream);

/* d_c[0] = sum_e E(rho_e) u_e^T K_e^0 u_e = u^T K u  (Eq. cmpc/cmpd, no 1/2);
 * d_c[1] = f^T u when d_f != NULL (d_f: [ndof] double).  Both FP64, summed in
 * a fixed order.  d_c: device array of 2 doubles. */
int soptx_compliance(soptx_pattern h, const soptx_material *m, const void *d_rho,
                     const double *d_u, const double *d_f, double *d_c, int32_t prec,
                     void *stream);

/* Fused soptx_sensitivity + soptx_compliance: one pass over the elements
 * computes u_e^T K_e^0 u_e once and writes both dc and c.  d_dc or d_c may
 * be NULL to skip that output. */
int soptx_evaluate(soptx_pattern h, const soptx_material *m, const void *d_rho,
                   const double *d_u, const double *d_f, void *d_dc, double *d_c, int32_t prec,
                   void *stream);

/* soptx_evaluate for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and results (bitwise) as soptx_evaluate, but the
 * block partials of the compliance live in a fixed device array of the
 * library (2 x 8192 doubles = 128 KiB per device, held from the library's
 * load until the process ends) instead of a workspace allocated on first
 * use: the call allocates nothing (no hipMalloc, no allocating library
 * routine).  Limit: with d_c != NULL, n_cells <= 8192 * 256 = 2,097,152;
 * larger meshes return SOPTX_E_SCRATCH before any device work (d_c == NULL
 * has no limit).  Every call on a device shares that device's array, which
 * keeps the last call's partials; each call overwrites every partial it
 * reads, so nothing needs clearing.  Calls that overlap on one device (on
 * different streams, or from different threads) race on the array and must
 * be serialized by the caller. */
int soptx_evaluate_noalloc(soptx_pattern h, const soptx_material *m, const void *d_rho,
                           const double *d_u, const double *d_f, void *d_dc, double *d_c,
                           int32_t prec, void *stream);

/* Reverse of soptx_assemble: for L = <Kbar, K(rho)>,
 * d_drho[e] = E'(rho_e) sum_ij Kbar[slot(e,i,j)] K_e^0[i,j],
 * where entries in a fixed row or column (d_dirichlet != NULL) are constants
 * of soptx_assemble and contribute nothing.  With Kbar = -u u^T restricted to
 * the pattern this equals dc (Appendix D).
 * d_Kbar: [nnz] double; d_drho: [n_cells] (double for SOPTX_FP64, float
 * otherwise).  The element matrices are contracted in FP64 for SOPTX_FP64 and
 * in FP32 (FP64 accumulation) otherwise. */
int soptx_assemble_backward(soptx_pattern h, const soptx_material *m, const void *d_rho,
                            const uint8_t *d_dirichlet, const double *d_Kbar, void *d_drho,
                            int32_t prec, void *stream);

/* y = K x for K in the pattern's CSR (d_K_vals: [nnz] double), x and y
 * [ndof] double (the matrix-vector product of the equilibrium system
 * K u = f, Sec. 2.2).  Each row is summed in a fixed order.  Asynchronous on
 * stream. */
int soptx_spmv(soptx_pattern h, const double *d_K_vals, const double *d_x, double *d_y, void *stream);

/* Build a pattern that also accepts Q1 elements whose map is not affine
 * (jittered or curved quadrilaterals and hexahedra), for the assembly with
 * per-quadrature-point geometry below: the same checks as
 * soptx_build_pattern, except that a non-affine Q1 element needs det J > 0
 * at every quadrature point (SOPTX_E_JACOBIAN otherwise).  Besides the
 * pattern it holds the node coordinates and, for every DIM x DIM block of K,
 * the list of its element contributions in ascending element order.  On a
 * handle of a mesh that has non-affine elements the affine-only calls
 * (soptx_assemble, soptx_evaluate and its variants, soptx_assemble_backward)
 * return SOPTX_E_NONAFFINE; pattern queries, soptx_apply_dirichlet,
 * soptx_spmv and soptx_pcg work on any handle.  SOPTX_HEX27 meshes (curved
 * or not, det J > 0 at every Gauss point of the 3 x 3 x 3 rule) are built
 * only here; on their handles the affine-only calls return
 * SOPTX_E_UNSUPPORTED_ELEM, and soptx_build_pattern refuses them with that
 * code. */
int soptx_build_pattern_general(const soptx_mesh *mesh, soptx_pattern *out, void *stream);

/* SIMP stiffness assembly (Sec. 2.1, Sec. 2.2) with the element matrices
 * integrated by the element's Gauss rule with J evaluated at every quadrature
 * point (Q1 quadrilaterals and hexahedra, affine or not, and Q2 hexahedra),
 * FP64: each element's
 * blocks E(rho_e) sum_q w_q |det J_q| L(g_i g_j^T), g = J_q^-T grad(phi) the
 * physical gradients, are formed in a workspace (n_cells nen^2 DIM^2 doubles
 * per (device, stream), allocated on first use), then every CSR block sums
 * its contributions in ascending element order.  d_rho: [n_cells] double;
 * d_dirichlet as in soptx_assemble (NULL: none); d_K_vals: [nnz].  Only for
 * handles of soptx_build_pattern_general (SOPTX_E_INVALID_ARG otherwise);
 * SOPTX_E_UNSUPPORTED_ELEM for simplices.  Asynchronous on stream. */
int soptx_assemble_general(soptx_pattern h, const soptx_material *m, const double *d_rho, const uint8_t *d_dirichlet,
                           double *d_K_vals, void *stream);

/* Element energies, sensitivities and compliance (Appendix D, Eq. cmpd) with
 * the Jacobian at every Gauss point (Q1, affine or not, and Q2 hexahedra; handles of
 * soptx_build_pattern_general), FP64: s_e = sum_q w_q |det J_q|
 * (lambda tr(eps)^2 + 2 mu eps:eps) = u_e^T K_e^0 u_e, d_dc[e] =
 * -p rho_e^(p-1) (E0 - Emin) s_e (d_dc may be NULL), d_c[0] = sum_e E(rho_e) s_e
 * and d_c[1] = f^T u when d_f is given (d_c may be NULL; not both NULL),
 * summed in a fixed order.  d_rho: [n_cells] double, d_u: [ndof].
 * SOPTX_E_INVALID_ARG for other handles, SOPTX_E_UNSUPPORTED_ELEM for
 * simplices.  Asynchronous on stream. */
int soptx_evaluate_general(soptx_pattern h, const soptx_material *m, const double *d_rho, const double *d_u,
                           const double *d_f, double *d_dc, double *d_c, void *stream);

/* Solve K u = f (Sec. 2.2) by conjugate gradients preconditioned by the
 * inverses of the DIM x DIM diagonal blocks of the nodes (node-block Jacobi;
 * the solver module's iterative solver, Sec. 3.2), for K
 * symmetric positive definite: assembled with a Dirichlet mask, f zero on
 * the fixed dofs.  d_u ([ndof] double) is the initial guess on entry and
 * the solution on return; d_f: [ndof] double.  Stops when
 * ||r_k|| <= rtol ||f|| (||r_0|| if f = 0; from u = 0 the two are the same)
 * for the recurrence residual, checked at the start and every 8 iterations,
 * or after max_iter iterations; *h_iters and *h_relres (host) give the count
 * and ||r_k|| / ||f|| (NaN after a breakdown, i.e. K not SPD).  A start
 * already within the tolerance returns after 0 iterations.  Synchronizes stream at those read-backs and at the start.  The
 * vectors live in a per-stream workspace of the library. */
int soptx_pcg(soptx_pattern h, const double *d_K_vals, const double *d_f, double *d_u, double rtol,
              int32_t max_iter, int32_t *h_iters, double *h_relres, void *stream);

/* Dirichlet boundary conditions bound once to a pattern (zero prescribed
 * values, Appendices A-C; the supports do not change during an optimisation,
 * Sec. 2.2).  h_mask: host [ndof] uint8, nonzero = fixed dof, read during the
 * call.  The handle holds, for the pattern's assembly plan, which stored
 * entries lie in a fixed row or column, so that soptx_step writes K with the
 * boundary conditions applied and no pass of its own: every fixed dof r gets
 * K[r,:] = 0, K[:,r] = 0, K[r,r] = 1, the same values as soptx_assemble with
 * that mask.  It is immutable and tied to h (destroy it before h); it
 * blocks until its device copies are made.  SOPTX_E_NONAFFINE /
 * SOPTX_E_UNSUPPORTED_ELEM on handles the affine calls refuse. */
typedef struct soptx_dirichlet_s *soptx_dirichlet;
int soptx_build_dirichlet(soptx_pattern h, const uint8_t *h_mask, soptx_dirichlet *out, void *stream);

/* Number of fixed dofs, and of plan groups whose blocks the mask touches
 * (either output may be NULL). */
int soptx_dirichlet_info(soptx_dirichlet bc, int64_t *n_fixed, int64_t *n_groups);

/* Release a Dirichlet handle (NULL is allowed). */
void soptx_destroy_dirichlet(soptx_dirichlet bc);

/* The whole per-iteration step of the paper's assembly and sensitivity path
 * (Sec. 2.1 SIMP, Sec. 2.2 Eq. cmpc/cmpd, Appendix D): d_K_vals =
 * soptx_assemble(rho) with the Dirichlet rows and columns of bc applied
 * while the assembly stages its blocks (bc NULL: none; no separate pass);
 * and, when d_u is given, the element energies s_e = u_e^T K_e^0 u_e of
 * soptx_evaluate: d_dc[e] = -E'(rho_e) s_e (d_dc may be NULL), d_c[0] =
 * sum_e E(rho_e) s_e and d_c[1] = f^T u (0 when d_f is NULL) (d_c may be
 * NULL).  d_u may be NULL only when d_dc and d_c are.  K is the same, value
 * for value, as soptx_assemble + the mask's Dirichlet step, and d_dc, d_c
 * are bit for bit those of soptx_evaluate, in both precision forms: the
 * energies run first (the kernel of soptx_evaluate), then the assembly,
 * which also adds the energy kernel's block partials of c in soptx_evaluate's
 * order (one launch fewer).  d_rho: [n_cells]; d_u, d_f: [ndof] double;
 * d_K_vals: [nnz]; d_dc: [n_cells]; d_c: 2 doubles.  Asynchronous on stream;
 * the compliance's partials live in a per-(device, stream) workspace
 * allocated on first use, so calls that overlap on one stream's workspace
 * are ordered by that stream. */
int soptx_step(soptx_pattern h, soptx_dirichlet bc, const soptx_material *m, const void *d_rho,
               const double *d_u, const double *d_f, double *d_K_vals, void *d_dc, double *d_c,
               int32_t prec, void *stream);

/* Release every device and host resource of h (NULL is allowed). */
void soptx_destroy_pattern(soptx_pattern h);

/* Static string for a status code. */
const char *soptx_status_string(int status);

/* Host-only: the reference tensor M[i][j][m][n] = int_ref d_m phi_i d_n phi_j
 * of an element type (Sec. 5.5), nen*nen*dim*dim doubles, by the chosen
 * method.  Touches no device. */
int soptx_reference_tensor(int32_t elem, int32_t ref_method, double *M_out);

/* Host-only validation of a mesh (the checks soptx_build_pattern runs before
 * any device work).  Touches no device. */
int soptx_validate_mesh(const soptx_mesh *mesh);

#ifdef __cplusplus
}
#endif
#endif /* SOPTX_H */
