// Kernel parameter blocks and launchers (device side in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace soptx {

constexpr int kF64 = SOPTX_FP64;
constexpr int kF32 = SOPTX_FP32;

struct AsmParams {
    const int32_t *grp_info;    // [G][kGrpInfo]: sig, n_nodes, elem_off, n_elem, n2l_off, flags
    const int32_t *grp_nodes;   // [G][64]
    const int32_t *grp_elems;   // per group, sorted element ids
    const uint16_t *grp_n2l;    // per group [K][64]: slot of the lane's k-th element
    const int32_t *grp_rows;    // [G][64][2]: first CSR slot of the node's rows, row length
    int os_window;              // one-shot variant: workgroups per window of XCD-local runs (multiple of 8)
    const int32_t *grp_rank_off;  // [G]: offset of the group's rank table, -1 = none (or NULL: no tables)
    const uint8_t *grp_rank;      // rank tables: [position][32] CSR position of a canonical position
    const int32_t *elem_by_rank;  // canonical-order plans: rank -> element, rho read through it (else null)
    const int32_t *sig_info;    // [S][4]: K, deg, pos_off, padded row-block size
    const int32_t *sig_pos_ptr;
    const int32_t *sig_contrib;
    const int32_t *sig_pairs;   // per signature (offset 2 pos_off): work items (pa, pb), -1 terminated
    const int32_t *sig_witems;  // [n][kWideInts]: wide work items
    const int32_t *sig_witem_ptr;  // [S + 1]
    const double *geo;
    const void *rho;
    const double *M;
    const float *M32;
    double *K;
    int64_t n_cells;
    int64_t n_groups;
    int n_cu;
    double E0, Emin, p;
    int ip;          // integer exponent, or -1
    double lam, mu;  // Lame constants at unit modulus (plane-stress lambda* in 2D)
    int kmax;
    int64_t stage;   // doubles of LDS stage needed by the largest group
    // the fused step (soptx_step) only; null in soptx_assemble
    const int32_t *bc_off;         // [G] offset of the group's Dirichlet bits, -1: none (null: no table)
    const uint8_t *bc_bits;        // per group [n_nodes][deg] bits of dirichlet_entry
    // the fused step with compliance: the energy kernel ran first; one wave
    // of workgroup 0 adds its block partials into fin_c[0..1] (null: none)
    const double *fin_partials;    // [2][fin_n]
    int fin_n;
    int fin_with_f;
    double *fin_c;
    // Q1 elements with per-point geometry (k_assemble_quad) only: per plan
    // column, sqrt(w_q |det J_q|) J_q^-1 at each Gauss point of the 2-point
    // rule on [0, 1]^DIM ([NQ][DIM][DIM][n_cells], entry (q, m, a) = d xi_m /
    // d x_a; point q at xi_m = (1 + 1/sqrt(3)) / 2 where bit m of q is set,
    // else (1 - 1/sqrt(3)) / 2)
    const double *qgeo;
};

struct EnergyParams {
    const int32_t *cells;
    const double *geo;
    const void *rho;
    const double *u;
    const double *qw;      // [NQ]
    const double *qgrad;   // [NQ][nen][dim]
    const float *qgrad32;  // [NQ][nen][dim]
    const double *cgrad;   // [nen][dim] reference gradients at the centroid
    const double *xref;    // [nen][dim] reference node coordinates
    void *dc;              // or null
    const double *f;       // [ndof] or null: f^T u as well
    int64_t ndof;
    double *partials;      // [2][grid] block partials of c and f^T u, or null (no compliance)
    int axis_aligned;      // every element has a diagonal J^-1 (the plan's groups all say so)
    int64_t n_cells;
    double E0, Emin, p;
    int ip;
    double lam, mu;
};

struct BwdParams {
    const int32_t *cells;
    const int32_t *row_ptr;
    const uint16_t *pos;
    const double *geo;
    const void *rho;
    const double *Kbar;
    const uint8_t *mask;
    const double *M;
    const float *M32;
    void *drho;
    int64_t n_cells;
    double E0, Emin, p;
    int ip;
    double lam, mu;
};

// fuse: the whole step (Dirichlet table, energies, dc, compliance partials)
hipError_t launch_assemble(int elem, int prec, const AsmParams &P, int64_t ngroups, hipStream_t st, bool fuse = false);
// which assembly kernel launch_assemble runs: -1 = chosen by the plan's shape
// (default), 0 = persistent (k_assemble), 1 = one-shot (k_assemble_os)
void set_assembly_variant(int v);
hipError_t launch_dirichlet(int dim, const int32_t *row_ptr, const int32_t *nb_tslot, const uint16_t *nb_tdeg,
                            const uint8_t *mask, double *K, int64_t ndof, hipStream_t st);
hipError_t launch_energy(int elem, int prec, const EnergyParams &P, hipStream_t st);
hipError_t launch_finalize(const double *partials, int n, int with_f, double *c, hipStream_t st);

// the allocation-free evaluate: its block partials live in a fixed device
// array of 2 x kNoAllocBlocks doubles (256 elements per block); the address
// of the current device's copy (device must be current)
constexpr int kNoAllocBlocks = 8192;
hipError_t noalloc_scratch(int device, double **out);

// solve (node-block Jacobi preconditioned CG); nb = neighbour lists, K's block structure
int64_t spmv_blocks(int dim, int64_t n_nodes);
hipError_t launch_spmv(int dim, const int32_t *row_ptr, const int32_t *nb, const double *K, const double *x,
                       double *y, double *xy_part, int64_t n_nodes, hipStream_t st);
int64_t cg_vec_blocks(int dim, int64_t ndof);
hipError_t launch_block_inv(int dim, const int32_t *row_ptr, const int32_t *nb, const double *K, double *binv,
                            int64_t n_nodes, hipStream_t st);
hipError_t launch_cg_vec(int dim, int mode, const double *f, double *u, double *r, double *z, double *p,
                         const double *q, const double *binv, const double *sc, double *part, int64_t ndof,
                         hipStream_t st);
hipError_t launch_cg_vec_fused(int dim, double *u, double *r, double *z, double *p, const double *q,
                               const double *binv, const double *pq_part, int n_pq, const double *sc,
                               double *part_out, int64_t ndof, hipStream_t st);
hipError_t launch_cg_p_fused(double *p, const double *z, const double *part, int nb, const double *sc_cur,
                             double *sc_next, int64_t n, hipStream_t st);
hipError_t launch_cg_p(double *p, const double *z, const double *sc, int64_t n, hipStream_t st);
hipError_t launch_cg_scalars(int what, const double *part, int n, double *sc, hipStream_t st);
hipError_t launch_backward(int elem, int prec, const BwdParams &P, hipStream_t st);

// per-quadrature-point assembly (non-affine Q1): element blocks, then a
// gather of every CSR block's contributions in ascending element order
struct GenParams {
    const int32_t *cells;
    const double *coords;
    const double *rho;
    const double *qw;
    const double *qgrad;  // [nq][nen][dim] reference gradients
    int64_t n_cells;
    int nq;
    double E0, Emin, p;
    int ip;
    double lam, mu;
    double *ke;  // [n_cells][nen][nen][dim][dim]
    const int32_t *gptr, *gent, *gnode, *row_ptr;
    double *K;
    int64_t n_blocks;
};
hipError_t launch_assemble_general(int elem, const GenParams &G, hipStream_t st);
// Q1 elements whose map is not affine, assembled in LDS from per-point
// geometry (P.qgeo, P.qref) on the plan's node groups, no element matrices in
// memory; FP64, no Dirichlet rows.  assemble_quad_fits: whether a plan's
// largest group fits the kernel's LDS (else the element-matrix path runs).
bool assemble_quad_fits(int elem, int64_t stage, int kmax);
hipError_t launch_assemble_quad(int elem, const AsmParams &P, int64_t ngroups, hipStream_t st);
// The same blocks with the partial sums in registers (k_assemble_point), for
// plans whose signatures have at most a fixed number of work items
// (max_items: the largest over the plan's signatures) and whose stage and
// gradients fit LDS.
bool assemble_point_fits(int elem, int64_t stage, int kmax, int max_items);
hipError_t launch_assemble_point(int elem, const AsmParams &P, int64_t ngroups, hipStream_t st);
// elements per block (and per c partial) of the Q2 hexahedron's energy kernel;
// the other elements take 256
constexpr int kEnergyWideElems = 16;
// element energies with per-quadrature-point geometry: dc and block partials
// of c and f^T u (as EnergyParams), FP64
struct GenEnergyParams {
    const int32_t *cells;
    const double *coords;
    const double *rho;
    const double *u;
    const double *qw;
    const double *qgrad;
    double *dc;        // or null
    const double *f;   // or null
    int64_t ndof;
    double *partials;  // [2][grid] or null
    int64_t n_cells;
    int nq;
    double E0, Emin, p;
    int ip;
    double lam, mu;
};
hipError_t launch_energy_general(int elem, const GenEnergyParams &P, hipStream_t st);

// filter step: H in CSR (int32 columns, FP64 weights), element measures v,
// row sums hsv_i = sum_j H_ij v_j and hs_i = sum_j H_ij; R rows per block
// (1..256), entries staged through LDS in chunks of kFilterChunk
constexpr int kFilterChunk = 2048;
struct FilterArgs {
    const int32_t *row_ptr;
    const int32_t *col;
    const double *w;
    const double *v;
    const double *hsv;
    const double *hs;
    int64_t n;
    // stencil form (S > 0): offsets [S][3] and weights over a grid of sizes N,
    // slowest axis first
    int S;
    const int32_t *sdel;
    const double *sw;
    int64_t N[3];
};
constexpr int kFilterStencilMax = 512;
hipError_t launch_filter_density(const FilterArgs &F, int R, const double *rho, double beta, double *rho_tilde,
                                 double *rho_bar, hipStream_t st);
hipError_t launch_filter_sensitivity(const FilterArgs &F, int R, const double *rho, const double *dc,
                                     double *dc_out, hipStream_t st);
// OC update: bisection subtree depth and node count per pass, block cap
constexpr int kOcDepth = 4;
constexpr int kOcNodes = (1 << kOcDepth) - 1;
constexpr int kOcMaxBlocks = 1024;
int oc_blocks(int64_t n);
hipError_t launch_oc_init(double *st, double lmax, hipStream_t s);
hipError_t launch_oc_pass(const double *rho, const double *dc, const double *dv, int64_t n, double move, double eta,
                          double vol_target, double tol, int max_steps, double *st, double *part, hipStream_t s);
hipError_t launch_oc_apply(const double *rho, const double *dc, const double *dv, int64_t n, double move, double eta,
                           double *st, double *out, double *part, hipStream_t s);
hipError_t launch_filter_backward(const FilterArgs &F, int R, const double *rho_tilde, double beta,
                                  const double *g, double *tmp, double *grad, hipStream_t st);

}  // namespace soptx
