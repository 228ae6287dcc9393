// C ABI of libsoptx: handle lifetime, argument validation, device uploads and
// kernel dispatch.  Every numeric step runs in the HIP kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/soptx.h"
#include "../../include/soptx_debug.h"
#include "host_util.h"
#include "internal.h"
#include "kernels.h"

using namespace soptx;

namespace soptx {

// Per-(device, stream, use) scratch; see host_util.h.
namespace {
struct Workspace {
    double *buf = nullptr;
    size_t n = 0;
};
std::mutex g_ws_mu;
std::map<std::tuple<int, hipStream_t, int>, Workspace> g_ws;
// Buffers replaced by larger ones.  They are kept, not freed: a HIP graph
// captured with a call on this stream holds their addresses, and a replay
// after a larger call must still find valid memory there (it also spares
// the host a synchronisation before the free)
std::vector<double *> g_ws_retired;
}  // namespace

int get_workspace(int device, hipStream_t st, size_t n, double **out, int use) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace &w = g_ws[std::make_tuple(device, st, use)];
    if (w.n < n) {
        if (w.buf) {
            try {
                g_ws_retired.push_back(w.buf);
            } catch (...) {
                return SOPTX_E_OOM;
            }
            w.buf = nullptr;
            w.n = 0;
        }
        size_t cap = n < 4096 ? 4096 : n;
        if (hipMalloc(&w.buf, cap * sizeof(double)) != hipSuccess) return SOPTX_E_OOM;
        w.n = cap;
    }
    *out = w.buf;
    return SOPTX_OK;
}

}  // namespace soptx


struct soptx_pattern_s {
    int elem = 0, dim = 0, nen = 0, ref_method = 0, device = 0, nq = 0;
    int64_t n_nodes = 0, n_cells = 0, ndof = 0, nnz = 0, ngroups = 0, nsig = 0;
    int emax = 0, kmax = 0;
    int64_t stage = 0;
    int32_t *row_ptr = nullptr, *col_idx = nullptr, *cells = nullptr;
    double *geo = nullptr;
    int32_t *grp_info = nullptr, *grp_nodes = nullptr, *grp_elems = nullptr;
    uint16_t *grp_n2l = nullptr;
    int32_t *grp_rows = nullptr;
    int32_t *grp_rank_off = nullptr;  // canonical-order plans only
    uint8_t *grp_rank = nullptr;
    int64_t n_rank_bytes = 0;
    int32_t *elem_by_rank = nullptr;  // canonical-order plans only: rank -> element
    double *geo_rank = nullptr;       // geo with its columns in rank order
    int n_cu = 0;
    int32_t *sig_info = nullptr, *sig_pos_ptr = nullptr, *sig_contrib = nullptr, *sig_pairs = nullptr;
    int32_t *sig_witems = nullptr, *sig_witem_ptr = nullptr;
    uint16_t *pos = nullptr, *nb_tdeg = nullptr;
    int32_t *nb_tslot = nullptr;
    int32_t *nb = nullptr;
    double *M = nullptr;
    float *M32 = nullptr;
    double *qw = nullptr, *qgrad = nullptr, *cgrad = nullptr, *xref = nullptr;
    // per-quadrature-point assembly (handles built by soptx_build_pattern_general)
    bool affine = true, general = false;
    double *coords = nullptr;
    int32_t *gptr = nullptr, *gent = nullptr, *gnode = nullptr;
    double *qgeo = nullptr;  // general Q1: per-point geometry of the row-block kernels
    int max_items = 0;       // largest number of work items of a signature
    float *qgrad32 = nullptr;
    soptx_pattern_stats stats{};
    std::vector<void *> allocs;
};

struct soptx_host_plan_s {
    HostPlan hp;
};

// A Dirichlet mask bound to a pattern: for every group of the plan whose
// blocks hold a fixed row or column, the offset of its bits (one byte per
// (node, neighbour position), see dirichlet_entry), -1 for the others.
struct soptx_dirichlet_s {
    soptx_pattern h = nullptr;
    int device = 0;
    int64_t n_fixed = 0, n_groups = 0;
    int32_t *off = nullptr;
    uint8_t *bits = nullptr;
    std::vector<void *> allocs;
    int64_t device_bytes = 0;
};

namespace {

template <class T>
int upload(soptx_pattern_s *h, const std::vector<T> &v, T **dst, hipStream_t st) {
    return upload_vector(h->allocs, v, dst, st, &h->stats.device_bytes);
}

void free_handle(soptx_pattern_s *h) {
    if (!h) return;
    for (void *p : h->allocs) (void)hipFree(p);
    delete h;
}

// the code an affine-only call returns on a handle with general elements
int not_affine(const soptx_pattern_s *h) {
    return h->elem == SOPTX_HEX27 ? SOPTX_E_UNSUPPORTED_ELEM : SOPTX_E_NONAFFINE;
}

int check_material(const soptx_material *m) {
    if (!m) return SOPTX_E_INVALID_ARG;
    if (!(m->E0 > m->Emin) || !(m->Emin >= 0.0) || !(m->nu > -1.0 && m->nu < 0.5) || !(m->p >= 1.0) ||
        !std::isfinite(m->E0) || !std::isfinite(m->p))
        return SOPTX_E_INVALID_ARG;
    return SOPTX_OK;
}

// Lame constants at unit modulus; 2D plane stress uses lambda* = nu/(1-nu^2)
void lame(const soptx_pattern_s *h, const soptx_material *m, double *lam, double *mu) {
    const double nu = m->nu;
    *mu = 1.0 / (2.0 * (1.0 + nu));
    if (h->dim == 2 && !m->plane_strain) *lam = nu / (1.0 - nu * nu);
    else *lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
}

int int_exponent(double p) {
    if (p == std::floor(p) && p >= 0.0 && p <= 16.0) return (int)p;
    return -1;
}

// SOPTX_BF16_FP32ACC is refused: bf16-rounded inputs miss the FP32 form's
// bound on K by two to three orders of magnitude
bool valid_prec(int32_t prec) { return prec == SOPTX_FP64 || prec == SOPTX_FP32; }

}  // namespace

extern "C" {

const char *soptx_status_string(int s) {
    switch (s) {
    case SOPTX_OK: return "ok";
    case SOPTX_E_INVALID_ARG: return "invalid argument";
    case SOPTX_E_UNSUPPORTED_ELEM: return "unsupported element type";
    case SOPTX_E_BAD_MESH: return "bad mesh (node index out of range or repeated in a cell)";
    case SOPTX_E_JACOBIAN: return "element with non-positive Jacobian determinant";
    case SOPTX_E_NONAFFINE: return "element map is not affine";
    case SOPTX_E_OVERFLOW: return "size exceeds the int32 index range";
    case SOPTX_E_OOM: return "out of memory";
    case SOPTX_E_DEVICE: return "HIP device or launch error";
    case SOPTX_E_SCRATCH: return "input exceeds the fixed scratch of an allocation-free call";
    default: return "unknown status";
    }
}

int soptx_validate_mesh(const soptx_mesh *mesh) { return validate_mesh(mesh); }

int soptx_reference_tensor(int32_t elem, int32_t ref_method, double *M_out) {
    if (!M_out) return SOPTX_E_INVALID_ARG;
    if (elem_dim(elem) < 0) return SOPTX_E_UNSUPPORTED_ELEM;
    return reference_tensor(elem, ref_method, M_out);
}

static int build_pattern(const soptx_mesh *mesh, int32_t ref_method, bool general, soptx_pattern *out,
                         void *stream) {
    if (!out) return SOPTX_E_INVALID_ARG;
    *out = nullptr;
    if (ref_method != SOPTX_REF_SYMBOLIC && ref_method != SOPTX_REF_QUADRATURE) return SOPTX_E_INVALID_ARG;
    HostPlan hp;
    int rc;
    try {
        rc = build_host_plan(mesh, hp, general);
    } catch (const std::bad_alloc &) {
        return SOPTX_E_OOM;
    } catch (...) {
        return SOPTX_E_INVALID_ARG;
    }
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    soptx_pattern_s *h = new (std::nothrow) soptx_pattern_s();
    if (!h) return SOPTX_E_OOM;
    try {
        h->elem = hp.elem; h->dim = hp.dim; h->nen = hp.nen; h->ref_method = ref_method;
        h->n_nodes = hp.n_nodes; h->n_cells = hp.n_cells; h->ndof = hp.ndof; h->nnz = hp.nnz;
        h->ngroups = hp.n_groups(); h->nsig = hp.n_sigs(); h->emax = hp.ne_max; h->kmax = hp.kmax; h->stage = hp.stage_max;
        h->affine = hp.affine; h->general = hp.general;
        for (int64_t sg = 0; sg < hp.n_sigs(); sg++) {
            const int deg = hp.sig_info[4 * sg + 1], posoff = hp.sig_info[4 * sg + 2];
            int n = 0;
            while (n <= deg && hp.sig_pairs[2 * (size_t)posoff + 2 * n] >= 0) n++;
            h->max_items = std::max({h->max_items, n, hp.sig_witem_ptr[sg + 1] - hp.sig_witem_ptr[sg]});
        }
        if (hipGetDevice(&h->device) != hipSuccess) { free_handle(h); return SOPTX_E_DEVICE; }
        if (hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess)
            h->n_cu = 0;
        // reference data
        const int nen = hp.nen, dim = hp.dim;
        std::vector<double> M((size_t)nen * nen * dim * dim);
        rc = reference_tensor(hp.elem, ref_method, M.data());
        if (rc) { free_handle(h); return rc; }
        std::vector<float> M32(M.begin(), M.end());
        std::vector<double> qw, qg;
        rc = reference_qp_grads(hp.elem, qw, qg);
        if (rc) { free_handle(h); return rc; }
        h->nq = (int)qw.size();
        std::vector<float> qg32(qg.begin(), qg.end());
        // centroid gradients and reference node coordinates (rigid-motion removal)
        std::vector<double> xref((size_t)nen * dim, 0.0), cg((size_t)nen * dim, 0.0);
        {
            static const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
            for (int i = 0; i < nen; i++) {
                if (hp.elem == SOPTX_QUAD4 || hp.elem == SOPTX_HEX8) {
                    for (int m = 0; m < dim; m++) xref[i * dim + m] = corner_bit(hp.elem, i, m);
                } else if (hp.elem == SOPTX_HEX27) {
                    for (int m = 0; m < dim; m++) xref[i * dim + m] = 0.5 * lattice_index(i, m);
                } else if (hp.elem == SOPTX_TRI3) {
                    if (i > 0) xref[i * dim + i - 1] = 1.0;
                } else {
                    auto v = [&](int vv, int m) { return (vv > 0 && vv - 1 == m) ? 1.0 : 0.0; };
                    for (int m = 0; m < 3; m++)
                        xref[i * dim + m] = i < 4 ? v(i, m) : 0.5 * (v(E[i - 4][0], m) + v(E[i - 4][1], m));
                }
            }
            // weighted mean of the quadrature-point gradients: the reference
            // gradient at the centroid (the rules are symmetric and the
            // gradients multilinear / affine)
            double wsum = 0.0;
            for (size_t q = 0; q < qw.size(); q++) wsum += qw[q];
            for (size_t q = 0; q < qw.size(); q++)
                for (int k = 0; k < nen * dim; k++) cg[k] += qw[q] / wsum * qg[q * nen * dim + k];
        }
        // pattern / plan uploads
        std::vector<int32_t> cells(mesh->cells, mesh->cells + (size_t)mesh->n_cells * nen);
        if ((rc = upload(h, hp.row_ptr, &h->row_ptr, st)) || (rc = upload(h, hp.col_idx, &h->col_idx, st)) ||
            (rc = upload(h, cells, &h->cells, st)) || (rc = upload(h, hp.geo, &h->geo, st))) {
            free_handle(h); return rc;
        }
        const int64_t base_bytes = h->stats.device_bytes;
        if ((rc = upload(h, hp.grp_info, &h->grp_info, st)) || (rc = upload(h, hp.grp_nodes, &h->grp_nodes, st)) ||
            (rc = upload(h, hp.grp_elems, &h->grp_elems, st)) || (rc = upload(h, hp.grp_n2l, &h->grp_n2l, st)) ||
            (rc = upload(h, hp.grp_rows, &h->grp_rows, st)) ||
            (hp.canonical && (rc = upload(h, hp.grp_rank_off, &h->grp_rank_off, st))) ||
            (hp.canonical && (rc = upload(h, hp.grp_rank, &h->grp_rank, st))) ||
            (hp.canonical && (rc = upload(h, hp.elem_by_rank, &h->elem_by_rank, st))) ||
            (hp.canonical && (rc = upload(h, hp.geo_rank, &h->geo_rank, st))) ||
            (rc = upload(h, hp.sig_info, &h->sig_info, st)) || (rc = upload(h, hp.sig_pos_ptr, &h->sig_pos_ptr, st)) ||
            (rc = upload(h, hp.sig_contrib, &h->sig_contrib, st)) || (rc = upload(h, hp.sig_pairs, &h->sig_pairs, st)) ||
            (rc = upload(h, hp.sig_witems, &h->sig_witems, st)) || (rc = upload(h, hp.sig_witem_ptr, &h->sig_witem_ptr, st))) {
            free_handle(h); return rc;
        }
        h->stats.plan_bytes = h->stats.device_bytes - base_bytes;
        h->n_rank_bytes = (int64_t)hp.grp_rank.size();
        if ((rc = upload(h, hp.pos, &h->pos, st)) || (rc = upload(h, hp.nb_tslot, &h->nb_tslot, st)) ||
            (rc = upload(h, hp.nb, &h->nb, st)) || (rc = upload(h, hp.nb_tdeg, &h->nb_tdeg, st)) || (rc = upload(h, M, &h->M, st)) ||
            (rc = upload(h, M32, &h->M32, st)) ||
            (rc = upload(h, qw, &h->qw, st)) || (rc = upload(h, qg, &h->qgrad, st)) ||
            (rc = upload(h, qg32, &h->qgrad32, st)) || (rc = upload(h, cg, &h->cgrad, st)) ||
            (rc = upload(h, xref, &h->xref, st))) {
            free_handle(h); return rc;
        }
        if (hp.general) {
            std::vector<double> xy(mesh->coords, mesh->coords + (size_t)mesh->n_nodes * dim);
            if ((rc = upload(h, xy, &h->coords, st)) || (rc = upload(h, hp.gptr, &h->gptr, st)) ||
                (rc = upload(h, hp.gent, &h->gent, st)) || (rc = upload(h, hp.gnode, &h->gnode, st)) ||
                (!hp.qgeo.empty() && (rc = upload(h, hp.qgeo, &h->qgeo, st)))) {
                free_handle(h);
                return rc;
            }
        }
        if (hipStreamSynchronize(st) != hipSuccess) { free_handle(h); return SOPTX_E_DEVICE; }
        const int64_t ncontrib = hp.n_cells * (int64_t)nen * nen;
        h->stats.ndof = hp.ndof; h->stats.nnz = hp.nnz; h->stats.n_cells = hp.n_cells; h->stats.n_nodes = hp.n_nodes;
        h->stats.n_groups = h->ngroups; h->stats.n_signatures = h->nsig; h->stats.n_contributions = ncontrib;
        for (int64_t g = 0; g < h->ngroups; g++)
            h->stats.n_groups_diag += (hp.grp_info[g * kGrpInfo + kGrpInfo - 1] & kGrpDiag) ? 1 : 0;
        for (int32_t ro : hp.grp_rank_off) h->stats.n_groups_ranked += ro >= 0 ? 1 : 0;
    } catch (const std::bad_alloc &) {
        free_handle(h);
        return SOPTX_E_OOM;
    }
    *out = h;
    return SOPTX_OK;
}

int soptx_build_pattern_ex(const soptx_mesh *mesh, int32_t ref_method, soptx_pattern *out, void *stream) {
    return build_pattern(mesh, ref_method, false, out, stream);
}

int soptx_build_pattern(const soptx_mesh *mesh, soptx_pattern *out, void *stream) {
    return soptx_build_pattern_ex(mesh, SOPTX_REF_SYMBOLIC, out, stream);
}

int soptx_build_pattern_general(const soptx_mesh *mesh, soptx_pattern *out, void *stream) {
    return build_pattern(mesh, SOPTX_REF_SYMBOLIC, true, out, stream);
}

static int asm_params(soptx_pattern h, const soptx_material *m, const void *d_rho, double *d_K_vals, int32_t prec,
                      hipStream_t st, AsmParams &P);
static int assemble_general_ke(soptx_pattern h, const soptx_material *m, const double *d_rho, double *d_K_vals,
                               hipStream_t st);

// which assembly general handles of Q1 elements run (soptx_debug_set_general_variant)
static std::atomic<int> g_general_variant{-1};

// the form of soptx_assemble_general on this handle: 1 = in LDS with the
// blocks' sums in registers (k_assemble_point), 2 = in LDS with the sums in
// the stage (k_assemble_quad), 0 = element matrices through memory
static int general_form(soptx_pattern h) {
    const int v = g_general_variant.load();
    if (!h->qgeo || v == 0) return 0;
    if (v != 1 && assemble_point_fits(h->elem, h->stage, h->kmax, h->max_items)) return 1;
    if (assemble_quad_fits(h->elem, h->stage, h->kmax)) return 2;
    return 0;
}

int soptx_assemble_general(soptx_pattern h, const soptx_material *m, const double *d_rho, const uint8_t *d_dirichlet,
                           double *d_K_vals, void *stream) {
    if (!h) return SOPTX_E_INVALID_ARG;
    if (!h->general) return SOPTX_E_INVALID_ARG;
    int rc = check_material(m);
    if (rc) return rc;
    if ((h->n_cells > 0 && !d_rho) || (h->nnz > 0 && !d_K_vals)) return SOPTX_E_INVALID_ARG;
    if (h->nnz == 0) return SOPTX_OK;
    if (h->elem != SOPTX_QUAD4 && h->elem != SOPTX_HEX8 && h->elem != SOPTX_HEX27) return SOPTX_E_UNSUPPORTED_ELEM;
    DeviceGuard dg(h->device);
    if (!dg.ok) return SOPTX_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int form = general_form(h);
    if (form) {
        AsmParams P{};
        if ((rc = asm_params(h, m, d_rho, d_K_vals, kF64, st, P))) return rc;
        P.qgeo = h->qgeo;
        const hipError_t e = form == 1 ? launch_assemble_point(h->elem, P, h->ngroups, st)
                                       : launch_assemble_quad(h->elem, P, h->ngroups, st);
        if (e != hipSuccess) return SOPTX_E_DEVICE;
    } else {
        rc = assemble_general_ke(h, m, d_rho, d_K_vals, st);
        if (rc) return rc;
    }
    if (d_dirichlet && launch_dirichlet(h->dim, h->row_ptr, h->nb_tslot, h->nb_tdeg, d_dirichlet, d_K_vals, h->ndof, st) != hipSuccess)
        return SOPTX_E_DEVICE;
    return SOPTX_OK;
}

// the element-matrix path: every element's matrix to memory, then one
// gather per block of K in ascending element order
static int assemble_general_ke(soptx_pattern h, const soptx_material *m, const double *d_rho, double *d_K_vals,
                               hipStream_t st) {
    int rc;
    const int nen = h->nen, dim = h->dim;
    double *ke = nullptr;
    rc = get_workspace(h->device, st, (size_t)h->n_cells * nen * nen * dim * dim, &ke, 4);
    if (rc) return rc;
    double lam, mu;
    lame(h, m, &lam, &mu);
    GenParams G{};
    G.cells = h->cells; G.coords = h->coords; G.rho = d_rho; G.qw = h->qw; G.qgrad = h->qgrad;
    G.n_cells = h->n_cells; G.nq = h->nq; G.E0 = m->E0; G.Emin = m->Emin; G.p = m->p; G.ip = int_exponent(m->p);
    G.lam = lam; G.mu = mu; G.ke = ke;
    G.gptr = h->gptr; G.gent = h->gent; G.gnode = h->gnode; G.row_ptr = h->row_ptr; G.K = d_K_vals;
    G.n_blocks = h->nnz / (dim * dim);
    if (launch_assemble_general(h->elem, G, st) != hipSuccess) return SOPTX_E_DEVICE;
    return SOPTX_OK;
}

int soptx_pattern_info(soptx_pattern h, int64_t *ndof, int64_t *nnz, const int32_t **d_row_ptr,
                       const int32_t **d_col_idx) {
    if (!h) return SOPTX_E_INVALID_ARG;
    if (ndof) *ndof = h->ndof;
    if (nnz) *nnz = h->nnz;
    if (d_row_ptr) *d_row_ptr = h->row_ptr;
    if (d_col_idx) *d_col_idx = h->col_idx;
    return SOPTX_OK;
}

int soptx_pattern_copy(soptx_pattern h, int32_t *h_row_ptr, int32_t *h_col_idx) {
    if (!h) return SOPTX_E_INVALID_ARG;
    DeviceGuard dg(h->device);
    if (!dg.ok) return SOPTX_E_DEVICE;
    if (h_row_ptr && hipMemcpy(h_row_ptr, h->row_ptr, sizeof(int32_t) * (h->ndof + 1), hipMemcpyDeviceToHost) != hipSuccess)
        return SOPTX_E_DEVICE;
    if (h_col_idx && h->nnz > 0 &&
        hipMemcpy(h_col_idx, h->col_idx, sizeof(int32_t) * h->nnz, hipMemcpyDeviceToHost) != hipSuccess)
        return SOPTX_E_DEVICE;
    return SOPTX_OK;
}

int soptx_pattern_stats_get(soptx_pattern h, soptx_pattern_stats *out) {
    if (!h || !out) return SOPTX_E_INVALID_ARG;
    *out = h->stats;
    return SOPTX_OK;
}

// Parameters of the assembly kernel.  A canonical-order plan reads its
// geometry in rank order (geo_rank, built with the plan) and the caller's
// densities through its rank -> element map.
static int asm_params(soptx_pattern h, const soptx_material *m, const void *d_rho, double *d_K_vals, int32_t prec,
                      hipStream_t st, AsmParams &P) {
    P.grp_info = h->grp_info; P.grp_nodes = h->grp_nodes; P.grp_elems = h->grp_elems; P.grp_n2l = h->grp_n2l;
    P.grp_rows = h->grp_rows; P.n_groups = h->ngroups; P.n_cu = h->n_cu;
    P.grp_rank_off = h->grp_rank_off; P.grp_rank = h->grp_rank;
    P.sig_info = h->sig_info; P.sig_pos_ptr = h->sig_pos_ptr; P.sig_contrib = h->sig_contrib;
    P.sig_pairs = h->sig_pairs; P.sig_witems = h->sig_witems; P.sig_witem_ptr = h->sig_witem_ptr;
    P.geo = h->geo; P.rho = d_rho;
    if (h->elem_by_rank) {
        // canonical order: the geometry columns in rank order (a copy made
        // with the plan); the densities read through the rank -> element map
        P.geo = h->geo_rank;
        P.elem_by_rank = h->elem_by_rank;
    }
    P.M = h->M; P.M32 = h->M32; P.K = d_K_vals;
    P.n_cells = h->n_cells; P.E0 = m->E0; P.Emin = m->Emin; P.p = m->p; P.ip = int_exponent(m->p);
    lame(h, m, &P.lam, &P.mu);
    P.kmax = h->kmax; P.stage = h->stage;
    return SOPTX_OK;
}

int soptx_assemble(soptx_pattern h, const soptx_material *m, const void *d_rho, const uint8_t *d_dirichlet,
                   double *d_K_vals, int32_t prec, void *stream) {
    if (!h || !valid_prec(prec)) return SOPTX_E_INVALID_ARG;
    if (!h->affine) return not_affine(h);
    int rc = check_material(m);
    if (rc) return rc;
    if ((h->n_cells > 0 && !d_rho) || (h->nnz > 0 && !d_K_vals)) return SOPTX_E_INVALID_ARG;
    if (h->nnz == 0) return SOPTX_OK;
    DeviceGuard dg(h->device);
    if (!dg.ok) return SOPTX_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    AsmParams P{};
    if ((rc = asm_params(h, m, d_rho, d_K_vals, prec, st, P))) return rc;
    if (launch_assemble(h->elem, prec, P, h->ngroups, st) != hipSuccess) return SOPTX_E_DEVICE;
    if (d_dirichlet && launch_dirichlet(h->dim, h->row_ptr, h->nb_tslot, h->nb_tdeg, d_dirichlet, d_K_vals, h->ndof, st) != hipSuccess)
        return SOPTX_E_DEVICE;
    return SOPTX_OK;
}

int soptx_apply_dirichlet(soptx_pattern h, const uint8_t *d_dirichlet, double *d_K_vals, void *stream) {
    if (!h || !d_dirichlet || (h->nnz > 0 && !d_K_vals)) return SOPTX_E_INVALID_ARG;
    if (h->nnz == 0) return SOPTX_OK;
    DeviceGuard dg(h->device);
    if (!dg.ok) return SOPTX_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (launch_dirichlet(h->dim, h->row_ptr, h->nb_tslot, h->nb_tdeg, d_dirichlet, d_K_vals, h->ndof, st) != hipSuccess)
        return SOPTX_E_DEVICE;
    return SOPTX_OK;
}

int soptx_spmv(soptx_pattern h, const double *d_K_vals, const double *d_x, double *d_y, void *stream) {
    if (!h || (h->nnz > 0 && (!d_K_vals || !d_x)) || (h->ndof > 0 && !d_y)) return SOPTX_E_INVALID_ARG;
    if (h->ndof == 0) return SOPTX_OK;
    DeviceGuard dg(h->device);
    if (!dg.ok) return SOPTX_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (launch_spmv(h->dim, h->row_ptr, h->nb, d_K_vals, d_x, d_y, nullptr, h->n_nodes, st) != hipSuccess)
        return SOPTX_E_DEVICE;
    return SOPTX_OK;
}

int soptx_pcg(soptx_pattern h, const double *d_K_vals, const double *d_f, double *d_u, double rtol,
              int32_t max_iter, int32_t *h_iters, double *h_relres, void *stream) {
    if (!h || !h_iters || !h_relres || max_iter < 0 || !(rtol >= 0.0)) return SOPTX_E_INVALID_ARG;
    if (h->ndof > 0 && (!d_K_vals || !d_f || !d_u)) return SOPTX_E_INVALID_ARG;
    *h_iters = 0;
    *h_relres = 0.0;
    if (h->ndof == 0) return SOPTX_OK;
    DeviceGuard dg(h->device);
    if (!dg.ok) return SOPTX_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = h->ndof;
    const int64_t nbv = cg_vec_blocks(h->dim, n);            // blocks of the vector kernels
    const int64_t nbs = spmv_blocks(h->dim, h->n_nodes);      // blocks of the SpMV
    const int64_t npart = std::max<int64_t>(3 * nbv, nbs);
    // Small systems fuse the scalar steps into the vector kernels: each of
    // their blocks re-reads the SpMV's partials, which pays while that is a few
    // MB (nbs * nbv doubles); the fused and separate steps give the same bits.
    const bool fused = nbs * nbv <= (int64_t)1 << 22;
    // r, z, p, q, the node blocks of the preconditioner (DIM doubles per dof),
    // partials, the fused path's second partials, 2 x 8 scalars (parity slots)
    double *ws = nullptr;
    int rc = get_workspace(h->device, st, (4 + (size_t)h->dim) * (size_t)n + (size_t)npart + 2 * (size_t)nbv + 16,
                           &ws, 1);
    if (rc) return rc;
    double *r = ws, *z = r + n, *p = z + n, *q = p + n, *binv = q + n, *part = binv + h->dim * n,
           *part2 = part + npart, *sc = part2 + 2 * nbv;
    int par = 0;  // fused path: the scalar slot sc + 8 par holds this iteration's r.z
    double hs[8];
    auto scalars = [&]() {
        if (hipMemcpyAsync(hs, sc + 8 * par, sizeof(hs), hipMemcpyDeviceToHost, st) != hipSuccess) return false;
        return hipStreamSynchronize(st) == hipSuccess;
    };
    // r = f - K u, z = B^-1 r, p = z
    if (launch_block_inv(h->dim, h->row_ptr, h->nb, d_K_vals, binv, h->n_nodes, st) != hipSuccess ||
        launch_spmv(h->dim, h->row_ptr, h->nb, d_K_vals, d_u, q, nullptr, h->n_nodes, st) != hipSuccess ||
        launch_cg_vec(h->dim, 0, d_f, d_u, r, z, p, q, binv, sc, part, n, st) != hipSuccess ||
        launch_cg_scalars(0, part, (int)nbv, sc, st) != hipSuccess ||
        launch_cg_scalars(3, part + 2 * nbv, (int)nbv, sc, st) != hipSuccess || !scalars())
        return SOPTX_E_DEVICE;
    const double rr0 = hs[4];
    if (!(rr0 > 0.0)) {  // u already solves the system (or the data hold a NaN)
        *h_relres = rr0 == 0.0 ? 0.0 : NAN;
        return SOPTX_OK;
    }
    // the residual is measured against ||f|| (against ||r_0|| when f = 0): from
    // u = 0 the two agree, and a start near the solution then needs fewer steps
    const double ref = hs[6] > 0.0 ? hs[6] : rr0;
    if (!(std::sqrt(rr0 / ref) > rtol)) {
        *h_relres = std::sqrt(rr0 / ref);
        return SOPTX_OK;
    }
    // the residual is read back every kCheck iterations
    constexpr int kCheck = 8;
    int it = 0;
    double rel = 1.0;
    while (it < max_iter) {
        if (launch_spmv(h->dim, h->row_ptr, h->nb, d_K_vals, p, q, part, h->n_nodes, st) != hipSuccess)
            return SOPTX_E_DEVICE;
        if (fused) {
            if (launch_cg_vec_fused(h->dim, d_u, r, z, p, q, binv, part, (int)nbs, sc + 8 * par, part2, n, st) !=
                    hipSuccess ||
                launch_cg_p_fused(p, z, part2, (int)nbv, sc + 8 * par, sc + 8 * (1 - par), n, st) != hipSuccess)
                return SOPTX_E_DEVICE;
            par = 1 - par;
        } else if (launch_cg_scalars(1, part, (int)nbs, sc, st) != hipSuccess ||
                   launch_cg_vec(h->dim, 1, d_f, d_u, r, z, p, q, binv, sc, part, n, st) != hipSuccess ||
                   launch_cg_scalars(2, part, (int)nbv, sc, st) != hipSuccess ||
                   launch_cg_p(p, z, sc, n, st) != hipSuccess) {
            return SOPTX_E_DEVICE;
        }
        it++;
        if (it % kCheck == 0 || it == max_iter) {
            if (!scalars()) return SOPTX_E_DEVICE;
            rel = std::sqrt(hs[3] / ref);
            if (!(rel > rtol)) break;  // converged, or broke down (NaN)
        }
    }
    *h_iters = it;
    *h_relres = rel;
    return SOPTX_OK;
}

// The element-energy kernel of soptx_evaluate and soptx_step: dc, and with
// d_c the fixed-order block partials of c and f^T u in the per-stream
// workspace or the fixed scratch (*ws, *nblk of each) for a finalize.
// Arguments are checked by the callers; the device is current.
static int launch_energies(soptx_pattern h, const soptx_material *m, const void *d_rho, const double *d_u,
                           const double *d_f, void *d_dc, double *d_c, int32_t prec, hipStream_t st, bool noalloc,
                           double **ws_out, int *nblk_out) {
    const int64_t nblk64 = std::max<int64_t>(1, (h->n_cells + 255) / 256);
    if (noalloc && d_c && nblk64 > kNoAllocBlocks) return SOPTX_E_SCRATCH;
    const int nblk = (int)nblk64;
    double *ws = nullptr;
    if (d_c) {
        // block partials of c, then of f^T u
        if (noalloc) {
            if (noalloc_scratch(h->device, &ws) != hipSuccess) return SOPTX_E_DEVICE;
        } else {
            const int rc = get_workspace(h->device, st, 2 * (size_t)nblk, &ws, 0);
            if (rc) return rc;
        }
    }
    EnergyParams P{};
    P.cells = h->cells; P.geo = h->geo; P.rho = d_rho; P.u = d_u;
    P.qw = h->qw; P.qgrad = h->qgrad; P.qgrad32 = h->qgrad32; P.cgrad = h->cgrad; P.xref = h->xref;
    P.dc = d_dc;
    P.f = d_c ? d_f : nullptr;
    P.ndof = h->ndof;
    P.partials = d_c ? ws : nullptr;
    P.axis_aligned = h->ngroups > 0 && h->stats.n_groups_diag == h->ngroups;
    P.n_cells = h->n_cells; P.E0 = m->E0; P.Emin = m->Emin; P.p = m->p; P.ip = int_exponent(m->p);
    lame(h, m, &P.lam, &P.mu);
    if (launch_energy(h->elem, prec, P, st) != hipSuccess) return SOPTX_E_DEVICE;
    *ws_out = ws;
    *nblk_out = nblk;
    return SOPTX_OK;
}

// soptx_evaluate and its allocation-free variant: the same kernels; the block
// partials of c go to the per-stream workspace or to the fixed scratch
static int evaluate_impl(soptx_pattern h, const soptx_material *m, const void *d_rho, const double *d_u,
                         const double *d_f, void *d_dc, double *d_c, int32_t prec, void *stream, bool noalloc) {
    if (!h || !valid_prec(prec)) return SOPTX_E_INVALID_ARG;
    if (!h->affine) return not_affine(h);
    int rc = check_material(m);
    if (rc) return rc;
    if (h->n_cells > 0 && (!d_rho || !d_u)) return SOPTX_E_INVALID_ARG;
    if (!d_dc && !d_c) return SOPTX_E_INVALID_ARG;
    if (noalloc && d_c && std::max<int64_t>(1, (h->n_cells + 255) / 256) > kNoAllocBlocks) return SOPTX_E_SCRATCH;
    DeviceGuard dg(h->device);
    if (!dg.ok) return SOPTX_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *ws = nullptr;
    int nblk = 0;
    if ((rc = launch_energies(h, m, d_rho, d_u, d_f, d_dc, d_c, prec, st, noalloc, &ws, &nblk))) return rc;
    if (d_c && launch_finalize(ws, nblk, d_f ? 1 : 0, d_c, st) != hipSuccess) return SOPTX_E_DEVICE;
    return SOPTX_OK;
}

int soptx_evaluate(soptx_pattern h, const soptx_material *m, const void *d_rho, const double *d_u,
                   const double *d_f, void *d_dc, double *d_c, int32_t prec, void *stream) {
    return evaluate_impl(h, m, d_rho, d_u, d_f, d_dc, d_c, prec, stream, false);
}

int soptx_evaluate_noalloc(soptx_pattern h, const soptx_material *m, const void *d_rho, const double *d_u,
                           const double *d_f, void *d_dc, double *d_c, int32_t prec, void *stream) {
    return evaluate_impl(h, m, d_rho, d_u, d_f, d_dc, d_c, prec, stream, true);
}

int soptx_evaluate_general(soptx_pattern h, const soptx_material *m, const double *d_rho, const double *d_u,
                           const double *d_f, double *d_dc, double *d_c, void *stream) {
    if (!h || !h->general) return SOPTX_E_INVALID_ARG;
    int rc = check_material(m);
    if (rc) return rc;
    if (h->n_cells > 0 && (!d_rho || !d_u)) return SOPTX_E_INVALID_ARG;
    if (!d_dc && !d_c) return SOPTX_E_INVALID_ARG;
    if (h->elem != SOPTX_QUAD4 && h->elem != SOPTX_HEX8 && h->elem != SOPTX_HEX27) return SOPTX_E_UNSUPPORTED_ELEM;
    DeviceGuard dg(h->device);
    if (!dg.ok) return SOPTX_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int per = h->elem == SOPTX_HEX27 ? kEnergyWideElems : 256;  // elements per partial
    const int nblk = std::max(1, (int)((h->n_cells + per - 1) / per));
    double *ws = nullptr;
    if (d_c) {
        rc = get_workspace(h->device, st, 2 * (size_t)nblk, &ws, 0);
        if (rc) return rc;
    }
    GenEnergyParams P{};
    P.cells = h->cells; P.coords = h->coords; P.rho = d_rho; P.u = d_u; P.qw = h->qw; P.qgrad = h->qgrad;
    P.dc = d_dc; P.f = d_c ? d_f : nullptr; P.ndof = h->ndof; P.partials = d_c ? ws : nullptr;
    P.n_cells = h->n_cells; P.nq = h->nq; P.E0 = m->E0; P.Emin = m->Emin; P.p = m->p; P.ip = int_exponent(m->p);
    lame(h, m, &P.lam, &P.mu);
    if (launch_energy_general(h->elem, P, st) != hipSuccess) return SOPTX_E_DEVICE;
    if (d_c && launch_finalize(ws, nblk, d_f ? 1 : 0, d_c, st) != hipSuccess) return SOPTX_E_DEVICE;
    return SOPTX_OK;
}

int soptx_sensitivity(soptx_pattern h, const soptx_material *m, const void *d_rho, const double *d_u,
                      void *d_dc, int32_t prec, void *stream) {
    if (h && h->n_cells > 0 && !d_dc) return SOPTX_E_INVALID_ARG;
    if (h && !h->affine) return not_affine(h);
    if (h && h->n_cells == 0) return (h && valid_prec(prec) && check_material(m) == 0) ? SOPTX_OK : SOPTX_E_INVALID_ARG;
    return soptx_evaluate(h, m, d_rho, d_u, nullptr, d_dc, nullptr, prec, stream);
}

int soptx_compliance(soptx_pattern h, const soptx_material *m, const void *d_rho, const double *d_u,
                     const double *d_f, double *d_c, int32_t prec, void *stream) {
    if (!d_c) return SOPTX_E_INVALID_ARG;
    return soptx_evaluate(h, m, d_rho, d_u, d_f, nullptr, d_c, prec, stream);
}

int soptx_assemble_backward(soptx_pattern h, const soptx_material *m, const void *d_rho,
                            const uint8_t *d_dirichlet, const double *d_Kbar, void *d_drho, int32_t prec,
                            void *stream) {
    if (!h || !valid_prec(prec)) return SOPTX_E_INVALID_ARG;
    if (!h->affine) return not_affine(h);
    int rc = check_material(m);
    if (rc) return rc;
    if (h->n_cells > 0 && (!d_rho || !d_Kbar || !d_drho)) return SOPTX_E_INVALID_ARG;
    if (h->n_cells == 0) return SOPTX_OK;
    DeviceGuard dg(h->device);
    if (!dg.ok) return SOPTX_E_DEVICE;
    BwdParams P{};
    P.cells = h->cells; P.row_ptr = h->row_ptr; P.pos = h->pos; P.geo = h->geo; P.rho = d_rho;
    P.Kbar = d_Kbar; P.M = h->M; P.M32 = h->M32; P.drho = d_drho; P.mask = d_dirichlet;
    P.n_cells = h->n_cells; P.E0 = m->E0; P.Emin = m->Emin; P.p = m->p; P.ip = int_exponent(m->p);
    lame(h, m, &P.lam, &P.mu);
    if (launch_backward(h->elem, prec, P, static_cast<hipStream_t>(stream)) != hipSuccess) return SOPTX_E_DEVICE;
    return SOPTX_OK;
}

int soptx_build_dirichlet(soptx_pattern h, const uint8_t *h_mask, soptx_dirichlet *out, void *stream) {
    if (!out) return SOPTX_E_INVALID_ARG;
    *out = nullptr;
    if (!h || (h->ndof > 0 && !h_mask)) return SOPTX_E_INVALID_ARG;
    if (!h->affine) return not_affine(h);
    DeviceGuard dg(h->device);
    if (!dg.ok) return SOPTX_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    soptx_dirichlet_s *bc = new (std::nothrow) soptx_dirichlet_s();
    if (!bc) return SOPTX_E_OOM;
    bc->h = h;
    bc->device = h->device;
    auto fail = [&](int code) {
        for (void *p : bc->allocs) (void)hipFree(p);
        delete bc;
        return code;
    };
    try {
        const int dim = h->dim, d2 = dim * dim;
        const int64_t G = h->ngroups;
        for (int64_t r = 0; r < h->ndof; r++) bc->n_fixed += h_mask[r] ? 1 : 0;
        // the plan's group tables and the neighbour lists, back from the device
        std::vector<int32_t> gi((size_t)G * kGrpInfo), si((size_t)h->nsig * 4), gn((size_t)G * kGroupNodes),
            rp((size_t)h->ndof + 1), nb((size_t)(h->nnz / d2));
        auto down = [&](std::vector<int32_t> &v, const int32_t *d) {
            return v.empty() || hipMemcpy(v.data(), d, v.size() * sizeof(int32_t), hipMemcpyDeviceToHost) == hipSuccess;
        };
        if (!down(gi, h->grp_info) || !down(si, h->sig_info) || !down(gn, h->grp_nodes) || !down(rp, h->row_ptr) ||
            !down(nb, h->nb))
            return fail(SOPTX_E_DEVICE);
        // canonical-order plans: the kernel's position p of a node is the CSR
        // position rank[p][lane] where the group has a rank table
        std::vector<int32_t> roff(h->grp_rank_off ? (size_t)G : 0);
        std::vector<uint8_t> rank(h->grp_rank ? (size_t)h->n_rank_bytes : 0);
        if (!down(roff, h->grp_rank_off) ||
            (!rank.empty() && hipMemcpy(rank.data(), h->grp_rank, rank.size(), hipMemcpyDeviceToHost) != hipSuccess))
            return fail(SOPTX_E_DEVICE);
        std::vector<int32_t> off((size_t)G, -1);
        std::vector<uint8_t> bits;
        if (bc->n_fixed > 0) {
            for (int64_t g = 0; g < G; g++) {
                const int nn = gi[(size_t)(kGrpInfo * g + 1)];
                const int deg = si[(size_t)(4 * gi[(size_t)(kGrpInfo * g)] + 1)];
                std::vector<uint8_t> gb((size_t)nn * deg, 0);
                bool any = false;
                for (int l = 0; l < nn; l++) {
                    const int64_t n = gn[(size_t)(g * kGroupNodes + l)];
                    int row = 0;
                    for (int a = 0; a < dim; a++) row |= h_mask[dim * n + a] ? 1 << a : 0;
                    const int64_t b0 = rp[(size_t)(dim * n)] / d2;
                    for (int p = 0; p < deg; p++) {
                        const int ro = roff.empty() ? -1 : roff[(size_t)g];
                        const int q = ro < 0 ? p : rank[(size_t)ro + (size_t)p * kGroupNodes + l];
                        const int64_t J = nb[(size_t)(b0 + q)];
                        int col = 0;
                        for (int c = 0; c < dim; c++) col |= h_mask[dim * J + c] ? 1 << (3 + c) : 0;
                        const int v = row | col | (J == n ? 64 : 0);
                        any = any || (row | col) != 0;
                        gb[(size_t)l * deg + p] = (uint8_t)v;
                    }
                }
                if (any) {
                    if (bits.size() + gb.size() >= (size_t)INT32_MAX) return fail(SOPTX_E_OVERFLOW);
                    off[(size_t)g] = (int32_t)bits.size();
                    bits.insert(bits.end(), gb.begin(), gb.end());
                    bc->n_groups++;
                }
            }
        }
        int rc;
        if ((rc = upload_vector(bc->allocs, off, &bc->off, st, &bc->device_bytes)) ||
            (rc = upload_vector(bc->allocs, bits, &bc->bits, st, &bc->device_bytes)))
            return fail(rc);
        if (hipStreamSynchronize(st) != hipSuccess) return fail(SOPTX_E_DEVICE);
    } catch (const std::bad_alloc &) {
        return fail(SOPTX_E_OOM);
    }
    *out = bc;
    return SOPTX_OK;
}

int soptx_dirichlet_info(soptx_dirichlet bc, int64_t *n_fixed, int64_t *n_groups) {
    if (!bc) return SOPTX_E_INVALID_ARG;
    if (n_fixed) *n_fixed = bc->n_fixed;
    if (n_groups) *n_groups = bc->n_groups;
    return SOPTX_OK;
}

void soptx_destroy_dirichlet(soptx_dirichlet bc) {
    if (!bc) return;
    DeviceGuard dg(bc->device);
    for (void *p : bc->allocs) (void)hipFree(p);
    delete bc;
}

int soptx_step(soptx_pattern h, soptx_dirichlet bc, const soptx_material *m, const void *d_rho, const double *d_u,
               const double *d_f, double *d_K_vals, void *d_dc, double *d_c, int32_t prec, void *stream) {
    if (!h || !valid_prec(prec)) return SOPTX_E_INVALID_ARG;
    if (!h->affine) return not_affine(h);
    int rc = check_material(m);
    if (rc) return rc;
    if (bc && bc->h != h) return SOPTX_E_INVALID_ARG;
    if ((h->n_cells > 0 && !d_rho) || (h->nnz > 0 && !d_K_vals)) return SOPTX_E_INVALID_ARG;
    if (h->n_cells > 0 && (d_dc || d_c) && !d_u) return SOPTX_E_INVALID_ARG;
    DeviceGuard dg(h->device);
    if (!dg.ok) return SOPTX_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // element energies and dc first (the kernel of soptx_evaluate; it does
    // not read K), so that the assembly kernel can add the partials of c in
    // the step where its store waves have nothing to store yet: the same
    // function and order as soptx_evaluate's finalize, one launch fewer
    double *ws = nullptr;
    int nblk = 0;
    if ((d_dc || d_c) && (rc = launch_energies(h, m, d_rho, d_u, d_f, d_dc, d_c, prec, st, false, &ws, &nblk)))
        return rc;
    // assembly with the Dirichlet table applied while the blocks are staged
    if (h->ngroups > 0) {
        AsmParams P{};
        if ((rc = asm_params(h, m, d_rho, d_K_vals, prec, st, P))) return rc;
        P.bc_off = (bc && bc->n_groups > 0) ? bc->off : nullptr;
        P.bc_bits = bc ? bc->bits : nullptr;
        if (d_c) {
            P.fin_partials = ws;
            P.fin_n = nblk;
            P.fin_with_f = d_f ? 1 : 0;
            P.fin_c = d_c;
        }
        if (launch_assemble(h->elem, prec, P, h->ngroups, st, true) != hipSuccess) return SOPTX_E_DEVICE;
    } else if (d_c && launch_finalize(ws, nblk, d_f ? 1 : 0, d_c, st) != hipSuccess) {
        return SOPTX_E_DEVICE;
    }
    return SOPTX_OK;
}

void soptx_destroy_pattern(soptx_pattern h) {
    if (!h) return;
    DeviceGuard dg(h->device);
    free_handle(h);
}

// ----------------------------------------------------------- host-only debug

int soptx_debug_set_general_variant(int32_t v) {
    if (v < -1 || v > 1) return SOPTX_E_INVALID_ARG;
    g_general_variant.store(v);
    return SOPTX_OK;
}

int soptx_debug_general_path(soptx_pattern h, int32_t *form) {
    if (!h || !form || !h->general) return SOPTX_E_INVALID_ARG;
    *form = general_form(h);
    return SOPTX_OK;
}

int soptx_debug_set_assembly_variant(int32_t v) {
    if (v < -1 || v > 1) return SOPTX_E_INVALID_ARG;
    set_assembly_variant(v);
    return SOPTX_OK;
}

int soptx_debug_host_plan(const soptx_mesh *mesh, soptx_host_plan *out) {
    return soptx_debug_host_plan_ex(mesh, 0, out);
}

int soptx_debug_host_plan_ex(const soptx_mesh *mesh, int32_t general, soptx_host_plan *out) {
    if (!out) return SOPTX_E_INVALID_ARG;
    *out = nullptr;
    soptx_host_plan_s *p = new (std::nothrow) soptx_host_plan_s();
    if (!p) return SOPTX_E_OOM;
    int rc;
    try {
        rc = build_host_plan(mesh, p->hp, general != 0);
    } catch (...) {
        rc = SOPTX_E_OOM;
    }
    if (rc) { delete p; return rc; }
    *out = p;
    return SOPTX_OK;
}

int soptx_debug_host_plan_array(soptx_host_plan p, const char *name, const void **data, int64_t *count,
                                int32_t *elem_bytes) {
    if (!p || !name || !data || !count || !elem_bytes) return SOPTX_E_INVALID_ARG;
    const HostPlan &hp = p->hp;
#define SOPTX_ARR(N)                                            \
    if (std::strcmp(name, #N) == 0) {                           \
        *data = hp.N.data();                                    \
        *count = (int64_t)hp.N.size();                         \
        *elem_bytes = (int32_t)sizeof(hp.N[0]);                 \
        return SOPTX_OK;                                        \
    }
    SOPTX_ARR(row_ptr) SOPTX_ARR(col_idx) SOPTX_ARR(geo) SOPTX_ARR(sig_info) SOPTX_ARR(sig_pos_ptr)
    SOPTX_ARR(sig_contrib) SOPTX_ARR(sig_pairs) SOPTX_ARR(sig_witems) SOPTX_ARR(sig_witem_ptr) SOPTX_ARR(grp_info) SOPTX_ARR(grp_nodes) SOPTX_ARR(grp_elems)
    SOPTX_ARR(grp_n2l) SOPTX_ARR(grp_rows) SOPTX_ARR(grp_rank_off) SOPTX_ARR(grp_rank) SOPTX_ARR(elem_by_rank)
    SOPTX_ARR(pos)
    SOPTX_ARR(nb_tslot) SOPTX_ARR(nb_tdeg)
    SOPTX_ARR(gptr) SOPTX_ARR(gent) SOPTX_ARR(gnode) SOPTX_ARR(qgeo)
#undef SOPTX_ARR
    return SOPTX_E_INVALID_ARG;
}

int soptx_debug_host_plan_scalars(soptx_host_plan p, int64_t *out8) {
    if (!p || !out8) return SOPTX_E_INVALID_ARG;
    const HostPlan &hp = p->hp;
    out8[0] = hp.ndof; out8[1] = hp.nnz; out8[2] = hp.n_groups(); out8[3] = hp.n_sigs();
    out8[4] = hp.emax; out8[5] = hp.kmax; out8[6] = hp.dim; out8[7] = hp.nen;
    return SOPTX_OK;
}

void soptx_debug_host_plan_free(soptx_host_plan p) { delete p; }

}  // extern "C"
