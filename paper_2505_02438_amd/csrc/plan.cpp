// Once-per-mesh host work: mesh validation, per-element geometry, the CSR
// pattern and the assembly plan (Sec. 3.2.2: invariant components are built
// once and reused across optimisation iterations).
#include <algorithm>
#include <atomic>
#include <array>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>
#include <unordered_map>
#include <unordered_set>

#include "../../include/soptx_debug.h"
#include "internal.h"

namespace soptx {

namespace {

int hw_threads() {
    unsigned n = std::thread::hardware_concurrency();
    if (n == 0) n = 4;
    if (n > 16) n = 16;
    return (int)n;
}

// Test hook: the next n worker chunks of parallel_for throw std::bad_alloc
// (soptx_debug_fail_workers), so that the failure path runs without
// exhausting memory.
std::atomic<int> g_fail_chunks{0};

// f(a, b) over chunks of [0, n) on up to hw_threads() threads.  An exception
// in a chunk is caught where it is thrown and reported by the return value
// (false); a thread that cannot be created leaves its chunk to the calling
// thread.  Every thread is joined before the return.
template <class F>
bool parallel_for(int64_t n, F &&f) {
    std::atomic<bool> failed{false};
    auto run = [&](int64_t a, int64_t b) {
        try {
            if (g_fail_chunks.load() > 0 && g_fail_chunks.fetch_sub(1) > 0) throw std::bad_alloc();
            f(a, b);
        } catch (...) {
            failed = true;
        }
    };
    const int T = hw_threads();
    if (n < 4096 || T <= 1) {
        run(0, n);
        return !failed;
    }
    std::vector<std::thread> th;
    try {
        th.reserve((size_t)T);
    } catch (...) {
    }
    const int64_t chunk = (n + T - 1) / T;
    for (int t = 1; t < T; t++) {
        const int64_t a = t * chunk, b = std::min(n, a + chunk);
        if (a >= b) break;
        try {
            th.emplace_back(run, a, b);
        } catch (...) {
            run(a, b);  // no thread available: the calling thread does the chunk
        }
    }
    run(0, std::min(n, chunk));
    for (auto &x : th) x.join();
    return !failed;
}

// det and inverse of a dim x dim row-major matrix J[a][m] = d x_a / d xi_m;
// G[m][a] = (J^-1)[m][a].
double inv_small(int dim, const double *J, double *G) {
    if (dim == 2) {
        double d = J[0] * J[3] - J[1] * J[2];
        G[0] = J[3] / d; G[1] = -J[1] / d; G[2] = -J[2] / d; G[3] = J[0] / d;
        return d;
    }
    double c00 = J[4] * J[8] - J[5] * J[7], c01 = J[5] * J[6] - J[3] * J[8], c02 = J[3] * J[7] - J[4] * J[6];
    double d = J[0] * c00 + J[1] * c01 + J[2] * c02;
    G[0] = c00 / d; G[1] = (J[2] * J[7] - J[1] * J[8]) / d; G[2] = (J[1] * J[5] - J[2] * J[4]) / d;
    G[3] = c01 / d; G[4] = (J[0] * J[8] - J[2] * J[6]) / d; G[5] = (J[2] * J[3] - J[0] * J[5]) / d;
    G[6] = c02 / d; G[7] = (J[1] * J[6] - J[0] * J[7]) / d; G[8] = (J[0] * J[4] - J[1] * J[3]) / d;
    return d;
}

// ---- contribution table of the per-quadrature-point assembly: block b of
// node n's neighbour q gets (e, i, j) for every element e holding both
// nodes, in ascending e (the order of a sequential element loop)
int general_table(const soptx_mesh *mesh, HostPlan &hp) {
    const int dim = hp.dim, nen = hp.nen;
    const int64_t NN = hp.n_nodes, NC = hp.n_cells;
    const int32_t *cells = mesh->cells;
    const int d2 = dim * dim;
    const int64_t nblk = hp.nnz / d2;
    if (NC * nen * nen >= INT32_MAX || nblk >= INT32_MAX) return SOPTX_E_OVERFLOW;
    auto blk = [&](int64_t e, int i, int j) {
        const int64_t I = cells[e * nen + i];
        return (int64_t)hp.row_ptr[(size_t)(dim * I)] / d2 + hp.pos[((size_t)e * nen + i) * nen + j];
    };
    hp.gptr.assign((size_t)nblk + 1, 0);
    for (int64_t e = 0; e < NC; e++)
        for (int i = 0; i < nen; i++)
            for (int j = 0; j < nen; j++) hp.gptr[(size_t)blk(e, i, j) + 1]++;
    for (int64_t b = 0; b < nblk; b++) hp.gptr[(size_t)b + 1] += hp.gptr[(size_t)b];
    hp.gent.assign((size_t)NC * nen * nen, 0);
    std::vector<int32_t> fill(hp.gptr.begin(), hp.gptr.end() - 1);
    for (int64_t e = 0; e < NC; e++)
        for (int i = 0; i < nen; i++)
            for (int j = 0; j < nen; j++)
                hp.gent[(size_t)fill[(size_t)blk(e, i, j)]++] = (int32_t)((e * nen + i) * nen + j);
    hp.gnode.assign((size_t)nblk, 0);
    for (int64_t n = 0; n < NN; n++) {
        const int64_t b0 = hp.row_ptr[(size_t)(dim * n)] / d2;
        const int64_t deg = (hp.row_ptr[(size_t)(dim * n + 1)] - hp.row_ptr[(size_t)(dim * n)]) / dim;
        for (int64_t q = 0; q < deg; q++) hp.gnode[(size_t)(b0 + q)] = (int32_t)n;
    }
    return SOPTX_OK;
}

}  // namespace

int validate_mesh(const soptx_mesh *mesh, bool allow_nonaffine, bool *affine) {
    if (affine) *affine = true;
    if (!mesh) return SOPTX_E_INVALID_ARG;
    const int dim = elem_dim(mesh->elem), nen = elem_nen(mesh->elem);
    if (dim < 0) return SOPTX_E_UNSUPPORTED_ELEM;
    // Q2 hexahedra run only through the per-quadrature-point assembly
    if (mesh->elem == SOPTX_HEX27 && !allow_nonaffine) return SOPTX_E_UNSUPPORTED_ELEM;
    if (mesh->dim != dim || mesh->n_nodes < 0 || mesh->n_cells < 0) return SOPTX_E_INVALID_ARG;
    if ((mesh->n_nodes > 0 && !mesh->coords) || (mesh->n_cells > 0 && !mesh->cells))
        return SOPTX_E_INVALID_ARG;
    if ((int64_t)dim * mesh->n_nodes >= INT32_MAX) return SOPTX_E_OVERFLOW;
    if (mesh->n_cells >= INT32_MAX / nen) return SOPTX_E_OVERFLOW;
    for (int64_t e = 0; e < mesh->n_cells; e++) {
        const int32_t *c = mesh->cells + e * nen;
        for (int i = 0; i < nen; i++) {
            if (c[i] < 0 || c[i] >= mesh->n_nodes) return SOPTX_E_BAD_MESH;
            for (int j = 0; j < i; j++)
                if (c[j] == c[i]) return SOPTX_E_BAD_MESH;
        }
    }
    // geometry: affine map, positive orientation
    std::vector<double> qw, qg;  // quadrature weights and reference gradients (non-affine Q1 only)
    for (int64_t e = 0; e < mesh->n_cells; e++) {
        const int32_t *c = mesh->cells + e * nen;
        auto X = [&](int i, int a) { return mesh->coords[(int64_t)c[i] * dim + a]; };
        // map-defining nodes: Q1 quad 0,1,3; Q1 and Q2 hex 0,1,3,4; simplices 0..dim
        int def[3];
        if (mesh->elem == SOPTX_QUAD4) { def[0] = 1; def[1] = 3; }
        else if (mesh->elem == SOPTX_HEX8 || mesh->elem == SOPTX_HEX27) { def[0] = 1; def[1] = 3; def[2] = 4; }
        else { for (int m = 0; m < dim; m++) def[m] = m + 1; }
        double J[9], G[9], scale = 0.0;
        for (int a = 0; a < dim; a++)
            for (int m = 0; m < dim; m++) {
                J[a * dim + m] = X(def[m], a) - X(0, a);
                scale = std::max(scale, std::fabs(J[a * dim + m]));
            }
        double det = inv_small(dim, J, G);
        // tensor-product elements may be general (Q1: not affine; Q2: curved)
        const bool q1 = mesh->elem == SOPTX_QUAD4 || mesh->elem == SOPTX_HEX8 || mesh->elem == SOPTX_HEX27;
        if (!(allow_nonaffine && q1) && (!(det > 0.0) || !std::isfinite(det))) return SOPTX_E_JACOBIAN;
        // every node must sit at the affine image of its reference position
        const double tol = 1e-10 * scale;
        bool is_affine = det > 0.0 && std::isfinite(det);
        for (int i = 0; i < nen; i++) {
            double xi[3] = {0, 0, 0};
            if (mesh->elem == SOPTX_QUAD4 || mesh->elem == SOPTX_HEX8) {
                for (int m = 0; m < dim; m++) xi[m] = corner_bit(mesh->elem, i, m);
            } else if (mesh->elem == SOPTX_HEX27) {
                for (int m = 0; m < dim; m++) xi[m] = 0.5 * lattice_index(i, m);
            } else if (mesh->elem == SOPTX_TRI3) {
                if (i > 0) xi[i - 1] = 1.0;
            } else {  // TET10: vertices then edge midpoints
                static const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
                auto vref = [](int v, double *o) { o[0] = o[1] = o[2] = 0.0; if (v > 0) o[v - 1] = 1.0; };
                if (i < 4) vref(i, xi);
                else {
                    double p[3], q[3];
                    vref(E[i - 4][0], p); vref(E[i - 4][1], q);
                    for (int m = 0; m < 3; m++) xi[m] = 0.5 * (p[m] + q[m]);
                }
            }
            for (int a = 0; a < dim; a++) {
                double x = X(0, a);
                for (int m = 0; m < dim; m++) x += J[a * dim + m] * xi[m];
                if (std::fabs(x - X(i, a)) > tol) is_affine = false;
            }
        }
        // a Q2 hexahedron always takes the Gauss-point check (and never the
        // affine-only calls)
        if (mesh->elem == SOPTX_HEX27 && affine) *affine = false;
        if (is_affine && mesh->elem != SOPTX_HEX27) continue;
        if (!(allow_nonaffine && q1)) return SOPTX_E_NONAFFINE;
        // a general element: det J > 0 at every quadrature point
        if (affine) *affine = false;
        if (qw.empty() && reference_qp_grads(mesh->elem, qw, qg)) return SOPTX_E_UNSUPPORTED_ELEM;
        for (size_t q = 0; q < qw.size(); q++) {
            double Jq[9], Gq[9];
            for (int a = 0; a < dim; a++)
                for (int m = 0; m < dim; m++) {
                    double t = 0.0;
                    for (int k = 0; k < nen; k++) t += X(k, a) * qg[(q * nen + k) * dim + m];
                    Jq[a * dim + m] = t;
                }
            const double dq = inv_small(dim, Jq, Gq);
            if (!(dq > 0.0) || !std::isfinite(dq)) return SOPTX_E_JACOBIAN;
        }
    }
    return SOPTX_OK;
}

// Canonical orders of nodes and elements: ranks that depend on the mesh's
// geometry and connectivity, not on how its nodes and elements are numbered.
// With h_a the lattice spacing along axis a (the median of |x_a(v) - x_a(w)|
// over pairs of vertices of one element that lie more than half the median
// element extent apart along a: unbiased under jitter) and o_a
// the phase of the vertex lattice along a (the circular mean of the element
// vertices' x_a modulo h_a, so that jittered lattice points round to their
// lattice positions):
//   node n: (q_0, ..., q_{d-1}), q_a = round(2 (x_a - o_a) / h_a) (edge
//     midpoints of quadratic elements fall on the odd values);
//   element e: the cell of its vertex centroid, c_a = floor((x_a - o_a) / h_a),
//     (c_0, ..., c_{d-1}), then the position of each of its vertices in that
//     cell, round(2 (x_a - o_a - c_a h_a) / h_a) clamped to 0..3, in local
//     vertex order (the elements of one cell differ there on a structured or
//     jittered grid);
// compared lexicographically (x slowest), ties by id.  A mesh numbered along
// its grid with x slowest gets its own numbering back; node_rank and
// elem_rank stay empty then.
static int canonical_orders(const soptx_mesh *mesh, std::vector<int32_t> &node_rank, std::vector<int32_t> &elem_rank) {
    node_rank.clear();
    elem_rank.clear();
    const int dim = elem_dim(mesh->elem), nen = elem_nen(mesh->elem);
    const int nv = mesh->elem == SOPTX_TRI3 ? 3 : mesh->elem == SOPTX_TET10 ? 4 : nen;
    const int64_t NN = mesh->n_nodes, NC = mesh->n_cells;
    if (NN == 0 || NC == 0 || nv > 8) return SOPTX_OK;
    const double *X = mesh->coords;
    const int32_t *cells = mesh->cells;
    double lo[3] = {0, 0, 0}, h[3] = {1, 1, 1};
    for (int a = 0; a < dim; a++) {
        std::vector<double> ext((size_t)NC);
        for (int64_t e = 0; e < NC; e++) {
            double mn = X[(int64_t)cells[e * nen] * dim + a], mx = mn;
            for (int v = 1; v < nv; v++) {
                const double x = X[(int64_t)cells[e * nen + v] * dim + a];
                mn = std::min(mn, x);
                mx = std::max(mx, x);
            }
            ext[(size_t)e] = mx - mn;
        }
        std::nth_element(ext.begin(), ext.begin() + NC / 2, ext.end());
        const double h0 = ext[(size_t)(NC / 2)];
        if (!(h0 > 0.0) || !std::isfinite(h0)) return SOPTX_OK;  // no usable spacing: keep the numbering
        // vertex pairs that span a cell along a, from at most ~2^17 elements
        std::vector<double> gap;
        const int64_t stride = std::max<int64_t>(1, NC >> 17);
        for (int64_t e = 0; e < NC; e += stride)
            for (int v = 0; v < nv; v++)
                for (int u = 0; u < v; u++) {
                    const double d = std::fabs(X[(int64_t)cells[e * nen + v] * dim + a] -
                                               X[(int64_t)cells[e * nen + u] * dim + a]);
                    if (d > 0.5 * h0) gap.push_back(d);
                }
        if (gap.empty()) return SOPTX_OK;
        std::nth_element(gap.begin(), gap.begin() + gap.size() / 2, gap.end());
        h[a] = gap[gap.size() / 2];
        // lattice phase: circular mean of the vertex coordinates modulo h
        const double w = 2.0 * M_PI / h[a];
        double sn = 0.0, cs = 0.0;
        for (int64_t e = 0; e < NC; e++)
            for (int v = 0; v < nv; v++) {
                const double x = X[(int64_t)cells[e * nen + v] * dim + a];
                sn += std::sin(w * x);
                cs += std::cos(w * x);
            }
        lo[a] = std::atan2(sn, cs) / w;
    }
    auto quant = [](double v) -> int64_t {
        if (!(std::fabs(v) < 4.0e18)) return v > 0 ? INT64_MAX / 2 : -INT64_MAX / 2;
        return (int64_t)std::floor(v);
    };
    // nodes
    std::vector<std::array<int64_t, 4>> nk((size_t)NN);
    for (int64_t n = 0; n < NN; n++) {
        nk[(size_t)n] = {0, 0, 0, n};
        for (int a = 0; a < dim; a++) nk[(size_t)n][a] = quant(2.0 * (X[n * dim + a] - lo[a]) / h[a] + 0.5);
    }
    std::sort(nk.begin(), nk.end());
    // elements
    std::vector<std::array<int64_t, 5>> ek((size_t)NC);
    for (int64_t e = 0; e < NC; e++) {
        double cen[3] = {0, 0, 0};
        for (int v = 0; v < nv; v++)
            for (int a = 0; a < dim; a++) cen[a] += X[(int64_t)cells[e * nen + v] * dim + a] / nv;
        int64_t c[3] = {0, 0, 0};
        for (int a = 0; a < dim; a++) c[a] = quant((cen[a] - lo[a]) / h[a]);
        uint64_t code = 0;
        for (int v = 0; v < nv; v++)
            for (int a = 0; a < dim; a++) {
                const double off = X[(int64_t)cells[e * nen + v] * dim + a] - lo[a] - (double)c[a] * h[a];
                int64_t r = quant(2.0 * off / h[a] + 0.5);
                r = std::max<int64_t>(0, std::min<int64_t>(3, r));
                code = (code << 2) | (uint64_t)r;
            }
        ek[(size_t)e] = {c[0], c[1], c[2], (int64_t)code, e};
    }
    std::sort(ek.begin(), ek.end());
    bool ident = true;
    for (int64_t n = 0; n < NN && ident; n++) ident = nk[(size_t)n][3] == n;
    for (int64_t e = 0; e < NC && ident; e++) ident = ek[(size_t)e][4] == e;
    if (ident) return SOPTX_OK;
    node_rank.assign((size_t)NN, 0);
    elem_rank.assign((size_t)NC, 0);
    for (int64_t r = 0; r < NN; r++) node_rank[(size_t)nk[(size_t)r][3]] = (int32_t)r;
    for (int64_t r = 0; r < NC; r++) elem_rank[(size_t)ek[(size_t)r][4]] = (int32_t)r;
    return SOPTX_OK;
}

// ---- per-point geometry of Q1 elements (the row-block assembly of general
// meshes), with the Gauss points of the 2-point rule per axis on [0, 1]^dim:
// point q at xi_m = gp where bit m of q is set, else gm, weight 1 / 2^dim.
// For every plan column (the element, or its rank in a canonical plan) and
// point q: sqrt(w_q |det J_q|) J_q^-1, J_q = sum_k x_k (grad phi_k(xi_q))^T;
// entry (q, m, a) = sqrt(w_q |det J_q|) d xi_m / d x_a at
// hp.qgeo[((q dim + m) dim + a) n_cells + column]
int quad_geometry(const soptx_mesh *mesh, HostPlan &hp) {
    const int dim = hp.dim, nen = hp.nen, d2 = dim * dim;
    const int nq = 1 << dim;
    if (nen != nq) return SOPTX_E_UNSUPPORTED_ELEM;
    const int64_t NC = hp.n_cells;
    const double gp = 0.78867513459481288225457439025098, gm = 0.21132486540518711774542560974902;
    const double w = 1.0 / nq;
    // d phi_k / d xi_m at point q: +-prod over the other axes n of gp where
    // node k's corner and point q agree on n, gm where they differ
    std::vector<double> rg((size_t)nq * nen * dim);
    for (int q = 0; q < nq; q++)
        for (int k = 0; k < nen; k++)
            for (int m = 0; m < dim; m++) {
                double t = 1.0;
                for (int n = 0; n < dim; n++)
                    if (n != m) t *= corner_bit(mesh->elem, k, n) == ((q >> n) & 1) ? gp : gm;
                rg[((size_t)q * nen + k) * dim + m] = corner_bit(mesh->elem, k, m) ? t : -t;
            }
    hp.qgeo.assign((size_t)nq * d2 * NC, 0.0);
    if (!parallel_for(NC, [&](int64_t a0, int64_t a1) {
        for (int64_t col = a0; col < a1; col++) {
            const int64_t e = hp.canonical ? hp.elem_by_rank[(size_t)col] : col;
            const int32_t *c = mesh->cells + e * nen;
            for (int q = 0; q < nq; q++) {
                double J[9], G[9];
                for (int a = 0; a < dim; a++)
                    for (int m = 0; m < dim; m++) {
                        double t = 0.0;
                        for (int k = 0; k < nen; k++)
                            t += mesh->coords[(int64_t)c[k] * dim + a] * rg[((size_t)q * nen + k) * dim + m];
                        J[a * dim + m] = t;
                    }
                const double det = inv_small(dim, J, G);
                const double s = std::sqrt(w * std::fabs(det));
                for (int x = 0; x < d2; x++) hp.qgeo[((size_t)q * d2 + x) * NC + col] = s * G[x];
            }
        }
    }))
        return SOPTX_E_OOM;
    return SOPTX_OK;
}

int build_host_plan(const soptx_mesh *mesh, HostPlan &hp, bool general) {
    int rc = validate_mesh(mesh, general, &hp.affine);
    if (rc) return rc;
    hp.general = general;
    const int dim = elem_dim(mesh->elem), nen = elem_nen(mesh->elem);
    const int64_t NN = mesh->n_nodes, NC = mesh->n_cells;
    hp.elem = mesh->elem; hp.dim = dim; hp.nen = nen;
    hp.n_nodes = NN; hp.n_cells = NC; hp.ndof = dim * NN;
    const int32_t *cells = mesh->cells;

    // ---- geometry (a1): G = J^-1 and det J per element, SoA
    hp.geo.assign((size_t)(dim * dim + 1) * NC, 0.0);
    if (!parallel_for(NC, [&](int64_t a0, int64_t a1) {
        for (int64_t e = a0; e < a1; e++) {
            const int32_t *c = cells + e * nen;
            int def[3];
            if (mesh->elem == SOPTX_QUAD4) { def[0] = 1; def[1] = 3; }
            else if (mesh->elem == SOPTX_HEX8 || mesh->elem == SOPTX_HEX27) { def[0] = 1; def[1] = 3; def[2] = 4; }
            else { for (int m = 0; m < dim; m++) def[m] = m + 1; }
            double J[9], G[9];
            for (int a = 0; a < dim; a++)
                for (int m = 0; m < dim; m++)
                    J[a * dim + m] = mesh->coords[(int64_t)c[def[m]] * dim + a] - mesh->coords[(int64_t)c[0] * dim + a];
            double det = inv_small(dim, J, G);
            for (int k = 0; k < dim * dim; k++) hp.geo[(size_t)k * NC + e] = G[k];
            hp.geo[(size_t)dim * dim * NC + e] = det;
        }
    }))
        return SOPTX_E_OOM;

    // ---- node -> (element, local index), elements ascending (counting sort)
    std::vector<int64_t> n2e_ptr(NN + 1, 0);
    for (int64_t e = 0; e < NC; e++)
        for (int i = 0; i < nen; i++) n2e_ptr[cells[e * nen + i] + 1]++;
    for (int64_t n = 0; n < NN; n++) n2e_ptr[n + 1] += n2e_ptr[n];
    std::vector<int32_t> n2e_e(n2e_ptr[NN]);
    std::vector<uint8_t> n2e_i(n2e_ptr[NN]);
    {
        std::vector<int64_t> fill(n2e_ptr.begin(), n2e_ptr.end() - 1);
        for (int64_t e = 0; e < NC; e++)
            for (int i = 0; i < nen; i++) {
                int64_t s = fill[cells[e * nen + i]]++;
                n2e_e[s] = (int32_t)e;
                n2e_i[s] = (uint8_t)i;
            }
    }

    // ---- neighbour lists (a2): sorted unique nodes of the adjacent elements
    std::vector<int64_t> deg(NN, 0);
    std::vector<int64_t> nb_ptr(NN + 1, 0);
    // first pass: degrees
    if (!parallel_for(NN, [&](int64_t a0, int64_t a1) {
        std::vector<int32_t> buf;
        for (int64_t n = a0; n < a1; n++) {
            buf.clear();
            for (int64_t s = n2e_ptr[n]; s < n2e_ptr[n + 1]; s++)
                for (int j = 0; j < nen; j++) buf.push_back(cells[(int64_t)n2e_e[s] * nen + j]);
            std::sort(buf.begin(), buf.end());
            deg[n] = std::unique(buf.begin(), buf.end()) - buf.begin();
        }
    }))
        return SOPTX_E_OOM;
    for (int64_t n = 0; n < NN; n++) nb_ptr[n + 1] = nb_ptr[n] + deg[n];
    const int64_t nnz = nb_ptr[NN] * dim * dim;
    if (nnz >= INT32_MAX) return SOPTX_E_OVERFLOW;
    for (int64_t n = 0; n < NN; n++)
        if (deg[n] > 65535) return SOPTX_E_OVERFLOW;
    hp.nnz = nnz;
    std::vector<int32_t> &nb = hp.nb;
    nb.assign(nb_ptr[NN], 0);
    if (!parallel_for(NN, [&](int64_t a0, int64_t a1) {
        std::vector<int32_t> buf;
        for (int64_t n = a0; n < a1; n++) {
            buf.clear();
            for (int64_t s = n2e_ptr[n]; s < n2e_ptr[n + 1]; s++)
                for (int j = 0; j < nen; j++) buf.push_back(cells[(int64_t)n2e_e[s] * nen + j]);
            std::sort(buf.begin(), buf.end());
            buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
            std::copy(buf.begin(), buf.end(), nb.begin() + nb_ptr[n]);
        }
    }))
        return SOPTX_E_OOM;

    // ---- CSR: rows dim*n+a hold dim*J+b for J in nb(n) ascending, b ascending
    hp.row_ptr.assign(hp.ndof + 1, 0);
    for (int64_t n = 0; n < NN; n++)
        for (int a = 0; a < dim; a++)
            hp.row_ptr[dim * n + a + 1] = (int32_t)(dim * dim * nb_ptr[n] + (a + 1) * dim * deg[n]);
    hp.col_idx.resize(nnz);
    if (!parallel_for(NN, [&](int64_t a0, int64_t a1) {
        for (int64_t n = a0; n < a1; n++)
            for (int a = 0; a < dim; a++) {
                int64_t o = hp.row_ptr[dim * n + a];
                for (int64_t k = nb_ptr[n]; k < nb_ptr[n + 1]; k++)
                    for (int b = 0; b < dim; b++) hp.col_idx[o++] = (int32_t)(dim * nb[k] + b);
            }
    }))
        return SOPTX_E_OOM;

    // ---- transposed slots: for J = nb(n)[q], the CSR slot of (row dim J,
    // column dim n) (n sits in nb(J): the neighbour relation is symmetric) and
    // the degree of J; the Dirichlet fix-up reaches the column entries of a
    // fixed dof through them
    hp.nb_tslot.assign(nb_ptr[NN], 0);
    hp.nb_tdeg.assign(nb_ptr[NN], 0);
    if (!parallel_for(NN, [&](int64_t a0, int64_t a1) {
        for (int64_t n = a0; n < a1; n++)
            for (int64_t k = nb_ptr[n]; k < nb_ptr[n + 1]; k++) {
                const int32_t J = nb[k];
                const int32_t *nj = nb.data() + nb_ptr[J];
                const int64_t t = std::lower_bound(nj, nj + deg[J], (int32_t)n) - nj;
                hp.nb_tslot[k] = (int32_t)(dim * dim * nb_ptr[J] + dim * t);
                hp.nb_tdeg[k] = (uint16_t)deg[J];
            }
    }))
        return SOPTX_E_OOM;

    if (mesh->elem == SOPTX_HEX27) {
        // only the per-quadrature-point assembly runs on these elements: the
        // position table alone, no signatures or groups
        hp.pos.assign((size_t)NC * nen * nen, 0);
        if (!parallel_for(NC, [&](int64_t a0, int64_t a1) {
            for (int64_t e = a0; e < a1; e++)
                for (int i = 0; i < nen; i++) {
                    const int64_t I = cells[e * nen + i];
                    const int32_t *nbn = nb.data() + nb_ptr[I];
                    for (int j = 0; j < nen; j++)
                        hp.pos[((size_t)e * nen + i) * nen + j] =
                            (uint16_t)(std::lower_bound(nbn, nbn + deg[I], cells[e * nen + j]) - nbn);
                }
        }))
            return SOPTX_E_OOM;
        return general_table(mesh, hp);
    }

    // ---- backward position table: position of cells[e][j] in the CSR
    // neighbour list of cells[e][i]
    hp.pos.assign((size_t)NC * nen * nen, 0);
    if (!parallel_for(NC, [&](int64_t a0, int64_t a1) {
        for (int64_t e = a0; e < a1; e++)
            for (int i = 0; i < nen; i++) {
                const int64_t I = cells[e * nen + i];
                const int32_t *nbn = nb.data() + nb_ptr[I];
                for (int j = 0; j < nen; j++)
                    hp.pos[((size_t)e * nen + i) * nen + j] =
                        (uint16_t)(std::lower_bound(nbn, nbn + deg[I], cells[e * nen + j]) - nbn);
            }
    }))
        return SOPTX_E_OOM;

    // ---- signatures.  In the given numbering a node's adjacent elements are
    // taken in ascending id and its neighbours in CSR order; in the canonical
    // order (canonical_orders) both follow ranks that do not depend on the
    // numbering, and nb_perm maps a canonical neighbour position to the CSR
    // one.  The canonical order is tried when the given numbering fragments
    // the plan (more than 64 signatures, fewer than 32 nodes per signature)
    // and kept when it at least halves the number of signatures.
    std::vector<int32_t> node_rank, elem_rank;
    bool canon = false;
    std::vector<uint8_t> nb_perm;  // [nb_ptr[NN]]: CSR position of canonical position pc of node n
    std::vector<int32_t> node_sig(NN, -1);
    std::vector<std::vector<int32_t>> sigs;  // canonical vectors
    auto signatures = [&](bool use_canon, std::vector<int32_t> &nsig_of, std::vector<std::vector<int32_t>> &sv_all) {
        std::unordered_map<uint64_t, std::vector<int32_t>> sig_by_hash;
        sv_all.clear();
        const int64_t CH = 1 << 16;
        for (int64_t c0 = 0; c0 < NN; c0 += CH) {
            int64_t c1 = std::min(NN, c0 + CH);
            std::vector<std::vector<int32_t>> sv(c1 - c0);
            std::vector<uint64_t> hv(c1 - c0);
            if (!parallel_for(c1 - c0, [&](int64_t a0, int64_t a1) {
                std::vector<std::array<int32_t, 4>> t;  // position, k, i, j
                std::vector<std::array<int64_t, 2>> ord;
                std::vector<int32_t> pc_of;
                for (int64_t x = a0; x < a1; x++) {
                    int64_t n = c0 + x;
                    const int32_t *nbn = nb.data() + nb_ptr[n];
                    const int64_t dg = deg[n];
                    const int K = (int)(n2e_ptr[n + 1] - n2e_ptr[n]);
                    if (use_canon) {
                        // canonical position of each CSR neighbour
                        ord.resize(dg);
                        for (int64_t q = 0; q < dg; q++) ord[q] = {node_rank[nbn[q]], q};
                        std::sort(ord.begin(), ord.end());
                        if ((int64_t)pc_of.size() < dg) pc_of.resize(dg);
                        for (int64_t r = 0; r < dg; r++) {
                            pc_of[ord[r][1]] = (int32_t)r;
                            nb_perm[nb_ptr[n] + r] = (uint8_t)ord[r][1];
                        }
                    }
                    t.clear();
                    for (int k = 0; k < K; k++) {
                        int64_t e = n2e_e[n2e_ptr[n] + k];
                        int i = n2e_i[n2e_ptr[n] + k];
                        for (int j = 0; j < nen; j++) {
                            int32_t J = cells[e * nen + j];
                            int p = (int)(std::lower_bound(nbn, nbn + dg, J) - nbn);
                            t.push_back({use_canon ? pc_of[p] : p, k, i, j});
                        }
                    }
                    std::sort(t.begin(), t.end());
                    std::vector<int32_t> &sg = sv[x];
                    sg.clear();
                    sg.push_back(K);
                    sg.push_back((int32_t)dg);
                    size_t q = 0;
                    for (int p = 0; p < dg; p++) {
                        size_t q0 = q;
                        while (q < t.size() && t[q][0] == p) q++;
                        sg.push_back((int32_t)(q - q0));
                        for (size_t r = q0; r < q; r++) sg.push_back((t[r][1] << 16) | (t[r][2] << 8) | t[r][3]);
                    }
                    uint64_t h = 1469598103934665603ull;
                    for (int32_t v : sg) { h ^= (uint32_t)v; h *= 1099511628211ull; }
                    hv[x] = h;
                }
            }))
                return false;
            for (int64_t x = 0; x < c1 - c0; x++) {
                auto &cand = sig_by_hash[hv[x]];
                int32_t id = -1;
                for (int32_t c : cand)
                    if (sv_all[c] == sv[x]) { id = c; break; }
                if (id < 0) {
                    id = (int32_t)sv_all.size();
                    sv_all.push_back(std::move(sv[x]));
                    cand.push_back(id);
                }
                nsig_of[c0 + x] = id;
            }
        }
        return true;
    };
    if (!signatures(false, node_sig, sigs)) return SOPTX_E_OOM;
    if (sigs.size() > 64 && (int64_t)sigs.size() * 32 > NN) {
        if ((rc = canonical_orders(mesh, node_rank, elem_rank))) return rc;
        canon = !node_rank.empty();
        for (int64_t n = 0; canon && n < NN; n++)
            if (deg[n] > 255) canon = false;  // canonical positions are stored in bytes
    }
    if (canon) {
        // the adjacent elements of every node in ascending rank
        std::vector<int32_t> e2(n2e_e);
        std::vector<uint8_t> i2(n2e_i);
        if (!parallel_for(NN, [&](int64_t a0, int64_t a1) {
            std::vector<std::array<int64_t, 3>> v;
            for (int64_t n = a0; n < a1; n++) {
                v.clear();
                for (int64_t s = n2e_ptr[n]; s < n2e_ptr[n + 1]; s++) v.push_back({elem_rank[e2[s]], e2[s], i2[s]});
                std::sort(v.begin(), v.end());
                for (size_t r = 0; r < v.size(); r++) {
                    e2[n2e_ptr[n] + r] = (int32_t)v[r][1];
                    i2[n2e_ptr[n] + r] = (uint8_t)v[r][2];
                }
            }
        }))
            return SOPTX_E_OOM;
        std::swap(e2, n2e_e);
        std::swap(i2, n2e_i);
        nb_perm.assign(nb_ptr[NN], 0);
        std::vector<int32_t> node_sig2(NN, -1);
        std::vector<std::vector<int32_t>> sigs2;
        if (!signatures(true, node_sig2, sigs2)) return SOPTX_E_OOM;
        if (2 * sigs2.size() <= sigs.size()) {
            node_sig.swap(node_sig2);
            sigs.swap(sigs2);
        } else {
            canon = false;
            std::swap(e2, n2e_e);
            std::swap(i2, n2e_i);
            nb_perm.clear();
        }
    }
    hp.canonical = canon;

    // ---- signature tables
    const int64_t nsig = (int64_t)sigs.size();
    hp.sig_info.assign(nsig * 4, 0);
    hp.sig_pos_ptr.clear();
    hp.sig_contrib.clear();
    hp.sig_pairs.clear();
    hp.kmax = 0;
    hp.blk_max = 0;
    for (int64_t s = 0; s < nsig; s++) {
        const auto &v = sigs[s];
        const int K = v[0], dg = v[1];
        hp.kmax = std::max(hp.kmax, K);
        // a node's row block (dim rows of dim*deg values), padded to an odd
        // number of doubles so that lanes (nodes) hit distinct LDS banks
        int blk = dim * dim * dg;
        if (blk % 2 == 0) blk += 1;
        hp.blk_max = std::max(hp.blk_max, blk);
        hp.sig_info[s * 4 + 0] = K;
        hp.sig_info[s * 4 + 1] = dg;
        hp.sig_info[s * 4 + 2] = (int32_t)hp.sig_pos_ptr.size();
        hp.sig_info[s * 4 + 3] = blk;
        size_t q = 2;
        for (int p = 0; p < dg; p++) {
            hp.sig_pos_ptr.push_back((int32_t)hp.sig_contrib.size());
            const int c = v[q++];
            for (int r = 0; r < c; r++) hp.sig_contrib.push_back(v[q++]);
        }
        hp.sig_pos_ptr.push_back((int32_t)hp.sig_contrib.size());
        // work items of the assembly kernel, one per wavefront (two halves):
        // a pair of positions (pa, pb), pb = -1 for a lone position, or a
        // position split between the halves (pb == pa).  Positions of
        // similar cost are paired; one that costs more than twice the next is
        // split.  Items are picked costliest first.
        const int32_t *pp = hp.sig_pos_ptr.data() + hp.sig_info[s * 4 + 2];
        auto cnt = [&](int p) { return pp[p + 1] - pp[p]; };
        std::vector<int32_t> order(dg);
        for (int p = 0; p < dg; p++) order[p] = p;
        std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return cnt(x) > cnt(y); });
        std::vector<std::array<int32_t, 3>> items;  // cost, pa, pb
        for (int i = 0; i < dg;) {
            const int p = order[i], c = cnt(p);
            if (i + 1 < dg && 2 * cnt(order[i + 1]) > c) {
                items.push_back({c, p, order[i + 1]});
                i += 2;
            } else if (c >= 2) {
                items.push_back({(c + 1) / 2, p, p});
                i += 1;
            } else {
                items.push_back({c, p, -1});
                i += 1;
            }
        }
        std::stable_sort(items.begin(), items.end(), [](const auto &x, const auto &y) { return x[0] > y[0]; });
        // 2 (deg + 1) entries per signature (offset 2 pos_off), -1 after the last item
        for (const auto &it : items) {
            hp.sig_pairs.push_back(it[1]);
            hp.sig_pairs.push_back(it[2]);
        }
        for (size_t k = items.size(); k < (size_t)dg + 1; k++) {
            hp.sig_pairs.push_back(-1);
            hp.sig_pairs.push_back(-1);
        }
    }
    // the assembly kernel reads contribution codes in chunks of 8 and reads
    // the second list of a pair as far as the first (longer) one: reads run
    // past a list's end by less than the longest list rounded up to 8 (the
    // codes there are not used).  A tail of that many zero codes keeps them
    // inside the table.
    {
        size_t longest = 0;
        for (size_t p = 0; p + 1 < hp.sig_pos_ptr.size(); p++)
            longest = std::max(longest, (size_t)(hp.sig_pos_ptr[p + 1] - hp.sig_pos_ptr[p]));
        hp.sig_contrib.insert(hp.sig_contrib.end(), std::max<size_t>(8, (longest + 7) / 8 * 8), 0);
    }
    if (hp.sig_contrib.size() >= (size_t)INT32_MAX) return SOPTX_E_OVERFLOW;

    // ---- groups: same-signature nodes in ascending order; at most kGroupNodes nodes,
    // at most kGroupElems distinct elements, and the group's row blocks must
    // fit the LDS stage of the assembly kernel
    hp.emax = kGroupElems;
    if (hp.kmax > kMaxAdjacent) return SOPTX_E_OVERFLOW;
    if ((int64_t)hp.blk_max * 8 > kStageBytes) return SOPTX_E_OVERFLOW;
    // one open group per signature; membership of its elements in a hash set
    // (groups of different signatures share elements)
    struct Open { std::vector<int32_t> nodes; std::vector<int32_t> elems; std::unordered_set<int32_t> in; };
    std::vector<Open> open(nsig);
    hp.grp_info.clear(); hp.grp_nodes.clear(); hp.grp_elems.clear(); hp.grp_n2l.clear(); hp.grp_rows.clear();
    hp.grp_rank_off.clear(); hp.grp_rank.clear();
    hp.stage_max = 0;
    struct Closed { int32_t sig; std::vector<int32_t> nodes, elems; };
    std::vector<Closed> closed;
    auto flush = [&](int64_t s) {
        Open &o = open[s];
        if (o.nodes.empty()) return;
        closed.push_back({(int32_t)s, std::move(o.nodes), std::move(o.elems)});
        o.nodes.clear();
        o.elems.clear();
        o.in.clear();
    };
    auto emit = [&](Closed &o) {
        const int64_t s = o.sig;
        const int K = hp.sig_info[s * 4 + 0];
        const int dg = hp.sig_info[s * 4 + 1];
        const int blk = hp.sig_info[s * 4 + 3];
        hp.stage_max = std::max<int64_t>(hp.stage_max, (int64_t)o.nodes.size() * blk);
        // elements sorted by id (by rank in the canonical order): for a fixed
        // k, neighbouring lanes then read neighbouring LDS slots on structured
        // meshes
        if (canon)
            std::sort(o.elems.begin(), o.elems.end(), [&](int32_t x, int32_t y) { return elem_rank[x] < elem_rank[y]; });
        else
            std::sort(o.elems.begin(), o.elems.end());
        // canonical order: the CSR position of each canonical neighbour
        // position, [position][lane], unless it is the position itself for
        // every node of the group
        int32_t roff = -1;
        if (canon) {
            bool ident = true;
            for (const int32_t n : o.nodes)
                for (int p = 0; p < dg && ident; p++) ident = nb_perm[nb_ptr[n] + p] == p;
            if (!ident) {
                roff = (int32_t)hp.grp_rank.size();
                for (int p = 0; p < dg; p++)
                    for (int l = 0; l < kGroupNodes; l++)
                        hp.grp_rank.push_back(l < (int)o.nodes.size() ? nb_perm[nb_ptr[o.nodes[l]] + p] : (uint8_t)p);
            }
        }
        if (canon) hp.grp_rank_off.push_back(roff);
        hp.grp_info.push_back((int32_t)s);
        hp.grp_info.push_back((int32_t)o.nodes.size());
        hp.grp_info.push_back((int32_t)hp.grp_elems.size());
        hp.grp_info.push_back((int32_t)o.elems.size());
        hp.grp_info.push_back((int32_t)hp.grp_n2l.size());
        // axis-aligned elements (off-diagonal entries of J^-1 exactly zero)
        // let the kernel form G'^T M G' from the diagonal alone
        bool diag = true;
        for (int32_t e : o.elems)
            for (int m = 0; m < dim && diag; m++)
                for (int a = 0; a < dim; a++)
                    if (m != a && hp.geo[(size_t)(m * dim + a) * NC + e] != 0.0) { diag = false; break; }
        hp.grp_info.push_back(diag ? kGrpDiag : 0);
        for (int l = 0; l < kGroupNodes; l++) hp.grp_nodes.push_back(l < (int)o.nodes.size() ? o.nodes[l] : -1);
        // canonical order: the elements by rank (the assembly reads their data
        // from arrays in rank order, geo_rank and the densities gathered so)
        for (int32_t e : o.elems) hp.grp_elems.push_back(canon ? elem_rank[e] : e);
        for (int k = 0; k < K; k++)
            for (int l = 0; l < kGroupNodes; l++) {
                const int ln = l < (int)o.nodes.size() ? l : 0;
                const int32_t e = n2e_e[n2e_ptr[o.nodes[ln]] + k];
                const int slot = (int)((canon ? std::lower_bound(o.elems.begin(), o.elems.end(), e,
                                                                 [&](int32_t x, int32_t y) {
                                                                     return elem_rank[x] < elem_rank[y];
                                                                 })
                                              : std::lower_bound(o.elems.begin(), o.elems.end(), e)) -
                                        o.elems.begin());
                hp.grp_n2l.push_back((uint16_t)slot);
            }
        for (int l = 0; l < kGroupNodes; l++) {
            if (l < (int)o.nodes.size()) {
                const int64_t n = o.nodes[l];
                hp.grp_rows.push_back(hp.row_ptr[dim * n]);
                hp.grp_rows.push_back(hp.row_ptr[dim * n + 1] - hp.row_ptr[dim * n]);
            } else {
                hp.grp_rows.push_back(0);
                hp.grp_rows.push_back(0);
            }
        }
    };
    // nodes in ascending id, or in ascending rank in the canonical order
    std::vector<int32_t> by_rank;
    if (canon) {
        by_rank.assign((size_t)NN, 0);
        for (int64_t n = 0; n < NN; n++) by_rank[(size_t)node_rank[n]] = (int32_t)n;
    }
    for (int64_t r = 0; r < NN; r++) {
        const int64_t n = canon ? by_rank[(size_t)r] : r;
        const int32_t s = node_sig[n];
        if (hp.sig_info[s * 4 + 1] == 0) continue;  // isolated node: empty rows
        Open &o = open[s];
        const int ncap = (int)std::min<int64_t>(kGroupNodes, kStageBytes / (8 * (int64_t)hp.sig_info[s * 4 + 3]));
        // count new elements this node would add
        int add = 0;
        for (int64_t q = n2e_ptr[n]; q < n2e_ptr[n + 1]; q++) add += o.in.count(n2e_e[q]) ? 0 : 1;
        if ((int)o.elems.size() + add > hp.emax || (int)o.nodes.size() >= ncap) flush(s);
        o.nodes.push_back((int32_t)n);
        for (int64_t q = n2e_ptr[n]; q < n2e_ptr[n + 1]; q++) {
            const int32_t e = n2e_e[q];
            if (o.in.insert(e).second) o.elems.push_back(e);
        }
    }
    for (int64_t s = 0; s < nsig; s++) flush(s);
    // groups in the order of their first node: the assembly kernel's
    // workgroups take consecutive groups at the same time, so the device
    // writes one contiguous window of K at a time and neighbouring groups
    // share element data in cache
    if (canon)
        std::sort(closed.begin(), closed.end(),
                  [&](const Closed &x, const Closed &y) { return node_rank[x.nodes[0]] < node_rank[y.nodes[0]]; });
    else
        std::sort(closed.begin(), closed.end(), [](const Closed &x, const Closed &y) { return x.nodes[0] < y.nodes[0]; });
    // ---- wide work items.  A signature whose groups hold at most N = 8 or 16
    // nodes would leave most lanes of a half-wave idle.  Its work items
    // instead cover P positions, each dealt round robin over Q phases
    // (contribution t to phase t mod Q), with P Q N = 64 lanes: lane =
    // (pp Q + q) N + node.  A position with c contributions gets the
    // smallest Q with ceil(c / Q) <= L, L = ceil(c_max / (64 / N)), so that
    // every lane runs at most L of them; positions with the same Q share
    // items, costliest first.
    std::vector<int> gmax(nsig, 0);
    for (const Closed &c : closed) gmax[c.sig] = std::max(gmax[c.sig], (int)c.nodes.size());
    std::vector<int> wideN(nsig, 32);
    hp.sig_witems.clear();
    hp.sig_witem_ptr.assign(1, 0);
    for (int64_t s = 0; s < nsig; s++) {
        if (gmax[s] > 0 && gmax[s] <= 16) wideN[s] = gmax[s] <= 8 ? 8 : 16;
        if (wideN[s] < 32) {
            const int PQ = 64 / wideN[s];
            const int dg = hp.sig_info[s * 4 + 1];
            const int32_t *pp = hp.sig_pos_ptr.data() + hp.sig_info[s * 4 + 2];
            int cmax = 1;
            for (int p = 0; p < dg; p++) cmax = std::max(cmax, pp[p + 1] - pp[p]);
            const int L = (cmax + PQ - 1) / PQ;
            std::vector<std::vector<int>> byQ(PQ + 1);
            for (int p = 0; p < dg; p++) {
                const int c = pp[p + 1] - pp[p];
                int Q = 1;
                while ((c + Q - 1) / Q > L) Q *= 2;
                byQ[Q].push_back(p);
            }
            std::vector<std::array<int32_t, kWideInts>> items;
            for (int Q = 1; Q <= PQ; Q *= 2) {
                auto &v = byQ[Q];
                std::stable_sort(v.begin(), v.end(), [&](int x, int y) { return pp[x + 1] - pp[x] > pp[y + 1] - pp[y]; });
                const int P = PQ / Q;
                for (size_t i = 0; i < v.size(); i += P) {
                    std::array<int32_t, kWideInts> r{};
                    r[0] = std::min<int>(P, (int)(v.size() - i));
                    r[1] = Q;
                    int T = 0;
                    for (int k = 0; k < 8; k++) {
                        const bool on = k < r[0];
                        const int p = on ? v[i + k] : -1;
                        const int c = on ? pp[p + 1] - pp[p] : 0;
                        r[8 + k] = p;
                        r[16 + k] = on ? pp[p] : 0;  // index into sig_contrib
                        r[24 + k] = c;
                        T = std::max(T, (c + Q - 1) / Q);
                    }
                    r[2] = T;
                    items.push_back(r);
                }
            }
            std::stable_sort(items.begin(), items.end(), [](const auto &x, const auto &y) { return x[2] > y[2]; });
            for (const auto &r : items) hp.sig_witems.insert(hp.sig_witems.end(), r.begin(), r.end());
        }
        hp.sig_witem_ptr.push_back((int32_t)(hp.sig_witems.size() / kWideInts));
    }
    for (Closed &c : closed) emit(c);
    // mark the groups of wide signatures
    for (int64_t g = 0; g < hp.n_groups(); g++) {
        const int N = wideN[hp.grp_info[kGrpInfo * g + 0]];
        if (N < 32) hp.grp_info[kGrpInfo * g + 5] |= (N == 8 ? 2 : 1) << kGrpWideShift;
    }
    hp.ne_max = 0;
    for (int64_t g = 0; g < hp.n_groups(); g++) hp.ne_max = std::max(hp.ne_max, hp.grp_info[kGrpInfo * g + 3]);
    if (canon) {
        // element data in rank order: the groups' elements are then as close
        // together in memory as on a mesh numbered along its grid
        hp.elem_by_rank.assign((size_t)NC, 0);
        for (int64_t e = 0; e < NC; e++) hp.elem_by_rank[(size_t)elem_rank[e]] = (int32_t)e;
        const int ng = dim * dim + 1;
        hp.geo_rank.assign(hp.geo.size(), 0.0);
        for (int c = 0; c < ng; c++)
            for (int64_t r = 0; r < NC; r++)
                hp.geo_rank[(size_t)c * NC + r] = hp.geo[(size_t)c * NC + hp.elem_by_rank[(size_t)r]];
    }
    if (hp.grp_elems.size() >= (size_t)INT32_MAX || hp.grp_n2l.size() >= (size_t)INT32_MAX ||
        hp.grp_rank.size() >= (size_t)INT32_MAX)
        return SOPTX_E_OVERFLOW;

    if (!general) return SOPTX_OK;
    rc = general_table(mesh, hp);
    if (rc || (mesh->elem != SOPTX_QUAD4 && mesh->elem != SOPTX_HEX8)) return rc;
    return quad_geometry(mesh, hp);
}

}  // namespace soptx

extern "C" int soptx_debug_fail_workers(int32_t n) {
    if (n < 0) return SOPTX_E_INVALID_ARG;
    soptx::g_fail_chunks.store(n);
    return SOPTX_OK;
}
