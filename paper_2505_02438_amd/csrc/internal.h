// Internal declarations shared by the host plan builder, the reference data,
// the HIP kernels and the C ABI of libsoptx.
#pragma once

#include <array>
#include <cstdint>
#include <vector>

#include "../../include/soptx.h"

namespace soptx {

constexpr int kGroupNodes = 32;    // nodes per assembly group = lanes of half a wavefront
constexpr int kGroupElems = 160;   // distinct elements per group (staged in LDS)
constexpr int kMaxAdjacent = 32;   // elements around one node (slot table entries per node)
constexpr int kStageBytes = 62208; // LDS for one group's row blocks (32 Q1-hex nodes x 243 values);
                                   // the assembly kernel holds two
constexpr int kMaxNen = 27;
// fields per group in grp_info, and the flag bits of its last field
constexpr int kGrpInfo = 6;
constexpr int kGrpDiag = 1;  // every element of the group has a diagonal J^-1 (axis-aligned)
// bits 1-2 of a group's flags: log2(32 / N) for a signature whose groups hold
// at most N = 8 or 16 nodes, run as wide work items (kGrpWideShift)
constexpr int kGrpWideShift = 1;
constexpr int kWideInts = 32;  // ints per wide work item: P, Q, T, 0 x 5, p[8], off[8], cnt[8]

inline int elem_dim(int elem) {
    switch (elem) {
    case SOPTX_QUAD4: case SOPTX_TRI3: return 2;
    case SOPTX_HEX8: case SOPTX_TET10: case SOPTX_HEX27: return 3;
    default: return -1;
    }
}
inline int elem_nen(int elem) {
    switch (elem) {
    case SOPTX_QUAD4: return 4;
    case SOPTX_TRI3: return 3;
    case SOPTX_HEX8: return 8;
    case SOPTX_TET10: return 10;
    case SOPTX_HEX27: return 27;
    default: return -1;
    }
}

int corner_bit(int elem, int i, int a);
int lattice_index(int i, int a);
void quadrature_rule(int elem, std::vector<double> &pts, std::vector<double> &wts);
int reference_tensor(int elem, int method, double *M);
int reference_qp_grads(int elem, std::vector<double> &wts, std::vector<double> &grads);

// Host-side result of the once-per-mesh build (pattern, geometry, plan).
//
// Assembly plan.  Nodes whose local connectivity is identical ("signature":
// number of adjacent elements K, number of neighbour nodes deg, and for each
// neighbour position p the ordered list of (k, i, j) = (index of the element
// in the node's ascending element list, local index of the node, local index
// of the neighbour)) are packed into groups of up to kGroupNodes.  The
// assembly kernel gives each half of a wavefront one neighbour position of
// the group's signature: lane = node within the half, and every lane of the
// half walks the same contributions.
struct HostPlan {
    int elem = 0, dim = 0, nen = 0;
    int64_t n_nodes = 0, n_cells = 0, ndof = 0, nnz = 0;
    std::vector<int32_t> row_ptr;  // [ndof+1]
    std::vector<int32_t> col_idx;  // [nnz]
    std::vector<double> geo;       // [(dim*dim+1)][n_cells]: G[m][a] = d xi_m / d x_a, then det J

    // signatures
    std::vector<int32_t> sig_info;     // [nsig][4]: K, deg, pos_off, blk (row-block doubles, odd)
    std::vector<int32_t> sig_pos_ptr;  // per signature deg+1 offsets into sig_contrib
    std::vector<int32_t> sig_contrib;  // (k << 16) | (i << 8) | j
    std::vector<int32_t> sig_pairs;    // per signature 2 (deg + 1) entries: work items (pa, pb), then -1
    // wide work items of the signatures whose groups hold at most 16 nodes:
    // signature s owns records sig_witem_ptr[s] .. sig_witem_ptr[s + 1]
    std::vector<int32_t> sig_witems;    // [n][kWideInts]
    std::vector<int32_t> sig_witem_ptr; // [nsig + 1]
    // groups
    std::vector<int32_t> grp_info;   // [ngroups][kGrpInfo]: sig, n_nodes, elem_off, n_elem, n2l_off, flags
    std::vector<int32_t> grp_nodes;  // [ngroups][kGroupNodes], -1 padded
    std::vector<int32_t> grp_elems;  // concatenated element ids, grp_info elem_off .. next
    std::vector<uint16_t> grp_n2l;   // per group K*kGroupNodes (k-major): slot of element k of lane's node
    std::vector<int32_t> grp_rows;   // [ngroups][kGroupNodes][2]: first CSR slot of the node's rows, row length
    // canonical order only (canonical = true): per group the offset of its
    // rank table in grp_rank, or -1 where every neighbour position is its CSR
    // position; a rank table holds, [position][kGroupNodes], the CSR position
    // of each canonical neighbour position of each node of the group
    bool canonical = false;
    std::vector<int32_t> grp_rank_off;  // [ngroups]
    std::vector<uint8_t> grp_rank;
    // canonical order only: grp_elems holds element ranks; elem_by_rank [n_cells]
    // maps a rank to its element, geo_rank is geo with its columns in rank order
    std::vector<int32_t> elem_by_rank;
    std::vector<double> geo_rank;
    // backward: position of cells[e][j] in the neighbour list of cells[e][i]
    std::vector<uint16_t> pos;       // [n_cells][nen][nen]
    // per node n and neighbour J = nb(n)[q] (offset row_ptr[dim n] / dim^2 + q):
    // the CSR slot of (row dim J, column dim n) and the degree of J
    std::vector<int32_t> nb_tslot;
    // per node n (offset row_ptr[dim n] / dim^2): its neighbour nodes, ascending
    std::vector<int32_t> nb;
    std::vector<uint16_t> nb_tdeg;
    int kmax = 0, emax = 0, ne_max = 0;  // emax: grouping limit; ne_max: largest group
    int blk_max = 0;                     // largest padded row block (doubles)
    int64_t stage_max = 0;               // largest group stage (doubles)
    bool affine = true;                  // every element map is affine
    // per-quadrature-point assembly (general = true): for every DIM x DIM block
    // b of K (b = row_ptr[dim n] / dim^2 + q for neighbour q of node n) its
    // contributions e * nen^2 + i * nen + j in ascending element order, and n
    bool general = false;
    std::vector<int32_t> gptr;   // [nnz / dim^2 + 1]
    std::vector<int32_t> gent;   // [n_cells * nen^2]
    std::vector<int32_t> gnode;  // [nnz / dim^2]
    // general Q1 elements only: per plan column (the element, or its rank in a
    // canonical plan) and Gauss point q, sqrt(w_q |det J_q|) J_q^-1,
    // [NQ][dim][dim][n_cells]
    std::vector<double> qgeo;
    int64_t n_groups() const { return (int64_t)grp_info.size() / kGrpInfo; }
    int64_t n_sigs() const { return (int64_t)sig_info.size() / 4; }
};

// allow_nonaffine: Q1 elements whose map is not affine are accepted when
// det J > 0 at every quadrature point (*affine is then set to false)
int validate_mesh(const soptx_mesh *mesh, bool allow_nonaffine = false, bool *affine = nullptr);
// general: also accept non-affine Q1 elements and build the contribution
// table of the per-quadrature-point assembly
int build_host_plan(const soptx_mesh *mesh, HostPlan &hp, bool general = false);

}  // namespace soptx
