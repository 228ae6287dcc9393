// Filter step of libsoptx (arXiv 2505.02438, Sec. 2.4; Sec. 3.2 filter
// module): the filter matrix H built once per mesh on the host, its device
// copy, and the C ABI of the filter products (kernels in filter.hip).
//
// Neighbourhood search: the centroids are binned into a uniform grid of cells
// of side h >= r_min, so every j with dist(i, j) < r_min lies in the 3^d
// cells around i's cell.  (The paper names a KD-tree; on the meshes of a
// topology-optimisation domain a uniform grid finds the same sets with less
// work.)  A row keeps the j with r_min - dist > 0, in ascending order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <unordered_map>
#include <cmath>
#include <new>
#include <thread>
#include <vector>

#include "../../include/soptx_debug.h"
#include "../../include/soptx_filter.h"
#include "host_util.h"
#include "internal.h"
#include "kernels.h"

using namespace soptx;

struct soptx_filter_s {
    int device = 0, dim = 0, rows_per_block = 1;
    int64_t n = 0, nnz = 0;
    int32_t *row_ptr = nullptr, *col = nullptr;
    double *w = nullptr, *v = nullptr, *hsv = nullptr, *hs = nullptr;
    // stencil form of H (S > 0): grid sizes in numbering order, offsets, weights
    int S = 0;
    int64_t N[3] = {1, 1, 1};
    int32_t *sdel = nullptr;
    double *sw = nullptr;
    std::vector<void *> allocs;
};

namespace {

// vertex (corner) nodes: Q1 quad 4, P1 triangle 3, Q1 hex 8, P2 tet 4, Q2 hex 8
// (its nodes 0-7)
int n_vertex(int elem) {
    switch (elem) {
    case SOPTX_QUAD4: return 4;
    case SOPTX_TRI3: return 3;
    case SOPTX_HEX8: case SOPTX_HEX27: return 8;
    case SOPTX_TET10: return 4;
    default: return -1;
    }
}

// Centroids (vertex mean, summed in local order) and measures: |det J| times
// the reference measure for an affine map, sum_q w_q |det J_q| over the Gauss
// points (exact for bilinear and trilinear maps) for a general Q1 element,
// and always for a Q2 hexahedron (3 x 3 x 3 points: det J has degree <= 5 in
// each variable, so the rule is exact for curved cells too).
void centroids_volumes(const soptx_mesh *m, std::vector<double> &c, std::vector<double> &v) {
    const int dim = m->dim, nen = elem_nen(m->elem), nv = n_vertex(m->elem);
    const int64_t n = m->n_cells;
    c.assign((size_t)n * dim, 0.0);
    v.assign((size_t)n, 0.0);
    std::vector<double> qw, qg;  // Gauss rule, for Q1 cells whose map is not affine
    // map-defining vertices and the reference measure
    int def[3];
    double ref = 1.0;
    if (m->elem == SOPTX_QUAD4) { def[0] = 1; def[1] = 3; }
    else if (m->elem == SOPTX_HEX8 || m->elem == SOPTX_HEX27) { def[0] = 1; def[1] = 3; def[2] = 4; }
    else { for (int a = 0; a < dim; a++) def[a] = a + 1; ref = dim == 2 ? 0.5 : 1.0 / 6.0; }
    for (int64_t e = 0; e < n; e++) {
        const int32_t *cell = m->cells + e * nen;
        auto X = [&](int i, int a) { return m->coords[(int64_t)cell[i] * dim + a]; };
        for (int a = 0; a < dim; a++) {
            double s = X(0, a);
            for (int i = 1; i < nv; i++) s += X(i, a);
            c[(size_t)e * dim + a] = s / nv;
        }
        double J[3][3];
        for (int a = 0; a < dim; a++)
            for (int b = 0; b < dim; b++) J[a][b] = X(def[b], a) - X(0, a);
        double det;
        if (dim == 2) det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        else
            det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                  J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        v[(size_t)e] = std::fabs(det) * ref;
        if (m->elem != SOPTX_QUAD4 && m->elem != SOPTX_HEX8 && m->elem != SOPTX_HEX27) continue;
        // a Q1 cell whose map is not affine: integrate |det J| at the Gauss points
        double scale = 0.0;
        for (int a = 0; a < dim; a++)
            for (int b = 0; b < dim; b++) scale = std::max(scale, std::fabs(J[a][b]));
        bool affine = m->elem != SOPTX_HEX27;
        for (int i = 0; i < nv && affine; i++)
            for (int a = 0; a < dim && affine; a++) {
                double x = X(0, a);
                for (int b = 0; b < dim; b++) x += J[a][b] * corner_bit(m->elem, i, b);
                affine = std::fabs(x - X(i, a)) <= 1e-10 * scale;
            }
        if (affine) continue;
        if (qw.empty()) reference_qp_grads(m->elem, qw, qg);
        double vol = 0.0;
        for (size_t q = 0; q < qw.size(); q++) {
            double Jq[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            for (int k = 0; k < nen; k++)
                for (int a = 0; a < dim; a++)
                    for (int b = 0; b < dim; b++) Jq[a][b] += X(k, a) * qg[(q * nen + k) * dim + b];
            const double dq = dim == 2 ? Jq[0][0] * Jq[1][1] - Jq[0][1] * Jq[1][0]
                                       : Jq[0][0] * (Jq[1][1] * Jq[2][2] - Jq[1][2] * Jq[2][1]) -
                                             Jq[0][1] * (Jq[1][0] * Jq[2][2] - Jq[1][2] * Jq[2][0]) +
                                             Jq[0][2] * (Jq[1][0] * Jq[2][1] - Jq[1][1] * Jq[2][0]);
            vol += qw[q] * std::fabs(dq);
        }
        v[(size_t)e] = vol;
    }
}

struct Rows {
    std::vector<int32_t> col;
    std::vector<double> w;
    std::vector<int64_t> cnt;
};

// rows [r0, r1) of H into out (per-row counts, then columns and weights)
void search_rows(int dim, const std::vector<double> &c, double rmin, const double *lo, double h, const int64_t *nc,
                 const std::vector<int64_t> &cell_ptr, const std::vector<int32_t> &cell_el, int64_t r0, int64_t r1,
                 Rows &out) {
    std::vector<std::pair<int32_t, double>> buf;
    for (int64_t i = r0; i < r1; i++) {
        buf.clear();
        const double *ci = &c[(size_t)i * dim];
        int64_t ic[3] = {0, 0, 0};
        for (int a = 0; a < dim; a++)
            ic[a] = std::min<int64_t>(nc[a] - 1, std::max<int64_t>(0, (int64_t)std::floor((ci[a] - lo[a]) / h)));
        const int64_t z0 = dim == 3 ? std::max<int64_t>(0, ic[2] - 1) : 0;
        const int64_t z1 = dim == 3 ? std::min<int64_t>(nc[2] - 1, ic[2] + 1) : 0;
        for (int64_t x = std::max<int64_t>(0, ic[0] - 1); x <= std::min<int64_t>(nc[0] - 1, ic[0] + 1); x++)
            for (int64_t y = std::max<int64_t>(0, ic[1] - 1); y <= std::min<int64_t>(nc[1] - 1, ic[1] + 1); y++)
                for (int64_t z = z0; z <= z1; z++) {
                    const int64_t cell = (x * nc[1] + y) * nc[2] + z;
                    for (int64_t q = cell_ptr[cell]; q < cell_ptr[cell + 1]; q++) {
                        const int32_t j = cell_el[q];
                        const double *cj = &c[(size_t)j * dim];
                        double d = ci[0] - cj[0];
                        double s = d * d;
                        for (int a = 1; a < dim; a++) {
                            d = ci[a] - cj[a];
                            s = s + d * d;
                        }
                        const double wij = rmin - std::sqrt(s);
                        if (wij > 0.0) buf.emplace_back(j, wij);
                    }
                }
        std::sort(buf.begin(), buf.end(), [](const auto &p, const auto &q) { return p.first < q.first; });
        out.cnt.push_back((int64_t)buf.size());
        for (const auto &p : buf) {
            out.col.push_back(p.first);
            out.w.push_back(p.second);
        }
    }
}

template <class T>
int upload(soptx_filter_s *h, const std::vector<T> &v, T **dst, hipStream_t st) {
    return upload_vector(h->allocs, v, dst, st);
}

void free_filter(soptx_filter_s *h) {
    if (!h) return;
    for (void *p : h->allocs) (void)hipFree(p);
    delete h;
}

FilterArgs args(const soptx_filter_s *h) {
    return FilterArgs{h->row_ptr, h->col, h->w, h->v, h->hsv, h->hs, h->n,
                      h->S, h->sdel, h->sw, {h->N[0], h->N[1], h->N[2]}};
}

int finish(hipError_t e) { return e == hipSuccess ? SOPTX_OK : SOPTX_E_DEVICE; }

struct HostFilter {
    int64_t n = 0;
    int dim = 0;
    std::vector<int32_t> row_ptr, col;
    std::vector<double> c, w, v, hsv, hs;
};

// H as a stencil: grid sizes N (slowest axis first, 1 for a missing axis),
// offsets del [S][3] in the same axis order sorted by linear offset, weights.
struct HostStencil {
    int64_t N[3] = {1, 1, 1};
    std::vector<int32_t> del;
    std::vector<double> w;
};

// H is a stencil when the elements form a structured grid numbered in
// lexicographic order of some axis order, and every row holds the same
// offsets (those inside the grid) with bitwise-equal weights.  Then the
// stencil, added in ascending offset order, reproduces each row's sum in
// ascending column order.
bool detect_stencil(const HostFilter &F, HostStencil &T) {
    const int64_t n = F.n;
    const int dim = F.dim;
    if (n == 0) return false;
    std::vector<double> uq[3];
    int64_t cnt[3] = {1, 1, 1};
    for (int a = 0; a < dim; a++) {
        uq[a].resize((size_t)n);
        for (int64_t e = 0; e < n; e++) uq[a][(size_t)e] = F.c[(size_t)e * dim + a];
        std::sort(uq[a].begin(), uq[a].end());
        uq[a].erase(std::unique(uq[a].begin(), uq[a].end()), uq[a].end());
        cnt[a] = (int64_t)uq[a].size();
    }
    if (cnt[0] * cnt[1] * cnt[2] != n) return false;
    std::vector<int64_t> g((size_t)n * 3, 0);
    for (int64_t e = 0; e < n; e++)
        for (int a = 0; a < dim; a++)
            g[(size_t)e * 3 + a] = std::lower_bound(uq[a].begin(), uq[a].end(), F.c[(size_t)e * dim + a]) - uq[a].begin();
    // axis orders, slowest first; a 2D grid gets a leading axis of size 1
    std::vector<std::array<int, 3>> perms;
    if (dim == 2) perms = {{-1, 0, 1}, {-1, 1, 0}};
    else perms = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int found = -1;
    for (size_t pi = 0; pi < perms.size() && found < 0; pi++) {
        const auto &p = perms[pi];
        int64_t N[3];
        for (int k = 0; k < 3; k++) N[k] = p[k] < 0 ? 1 : cnt[p[k]];
        bool ok = true;
        for (int64_t e = 0; e < n && ok; e++) {
            int64_t co[3];
            for (int k = 0; k < 3; k++) co[k] = p[k] < 0 ? 0 : g[(size_t)e * 3 + p[k]];
            ok = (co[0] * N[1] + co[1]) * N[2] + co[2] == e;
        }
        if (ok) {
            found = (int)pi;
            for (int k = 0; k < 3; k++) T.N[k] = N[k];
        }
    }
    if (found < 0) return false;
    const int64_t N1 = T.N[1], N2 = T.N[2];
    auto coords = [&](int64_t e, int64_t *co) {
        co[2] = e % N2;
        co[1] = (e / N2) % N1;
        co[0] = e / (N1 * N2);
    };
    // offsets and weights over every entry; key: the offset in a grid of
    // sizes 2N - 1 (unique for offsets between two points of the grid)
    const int64_t M1 = 2 * N1 + 1, M2 = 2 * N2 + 1;
    std::unordered_map<int64_t, size_t> idx;
    std::vector<std::pair<std::array<int64_t, 3>, double>> st;
    for (int64_t i = 0; i < n; i++) {
        int64_t ci[3], cj[3];
        coords(i, ci);
        for (int32_t k = F.row_ptr[(size_t)i]; k < F.row_ptr[(size_t)i + 1]; k++) {
            coords(F.col[(size_t)k], cj);
            const std::array<int64_t, 3> d{cj[0] - ci[0], cj[1] - ci[1], cj[2] - ci[2]};
            const int64_t key = (d[0] * M1 + d[1]) * M2 + d[2];
            auto it = idx.find(key);
            if (it == idx.end()) {
                if ((int)st.size() >= kFilterStencilMax) return false;
                idx.emplace(key, st.size());
                st.push_back({d, F.w[(size_t)k]});
            } else if (!(st[it->second].second == F.w[(size_t)k])) {
                return false;
            }
        }
    }
    // every row holds exactly the offsets that land inside the grid (its
    // entries are distinct offsets of the stencil, so equal counts suffice)
    for (int64_t i = 0; i < n; i++) {
        int64_t ci[3];
        coords(i, ci);
        int64_t in = 0;
        for (const auto &kv : st) {
            bool inside = true;
            for (int k = 0; k < 3; k++) {
                const int64_t x = ci[k] + kv.first[k];
                inside = inside && x >= 0 && x < T.N[k];
            }
            in += inside;
        }
        if (in != F.row_ptr[(size_t)i + 1] - F.row_ptr[(size_t)i]) return false;
    }
    // ascending linear offset = ascending column within every row
    std::vector<std::pair<int64_t, std::pair<std::array<int64_t, 3>, double>>> ent;
    for (const auto &kv : st) ent.push_back({(kv.first[0] * N1 + kv.first[1]) * N2 + kv.first[2], kv});
    // distinct offsets within the grid have distinct linear offsets
    std::sort(ent.begin(), ent.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    for (const auto &e : ent) {
        for (int k = 0; k < 3; k++) T.del.push_back((int32_t)e.second.first[k]);
        T.w.push_back(e.second.second);
    }
    return true;
}

int build_filter_host(const soptx_mesh *mesh, double rmin, HostFilter &F) {
    if (!(rmin > 0.0) || !std::isfinite(rmin)) return SOPTX_E_INVALID_ARG;
    int rc = validate_mesh(mesh, true);  // general Q1 cells too (det J > 0 at the Gauss points)
    if (rc) return rc;
    const int dim = mesh->dim;
    const int64_t n = mesh->n_cells;
    F.n = n;
    F.dim = dim;
    std::vector<double> &c = F.c;
    std::vector<double> &v = F.v, &w = F.w, &hsv = F.hsv, &hs = F.hs;
    std::vector<int32_t> &row_ptr = F.row_ptr, &col = F.col;
    row_ptr.assign((size_t)n + 1, 0);
    hsv.assign((size_t)n, 0.0);
    hs.assign((size_t)n, 0.0);
    try {
        centroids_volumes(mesh, c, v);
        // bounding box and cell grid (side h >= rmin, at most ~2 cells per element)
        double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int a = 0; a < dim; a++) {
            lo[a] = n ? c[a] : 0.0;
            hi[a] = lo[a];
        }
        for (int64_t e = 0; e < n; e++)
            for (int a = 0; a < dim; a++) {
                lo[a] = std::min(lo[a], c[(size_t)e * dim + a]);
                hi[a] = std::max(hi[a], c[(size_t)e * dim + a]);
            }
        double h = rmin;
        int64_t nc[3] = {1, 1, 1};
        for (int doubling = 0;; doubling++) {
            double cells = 1.0;
            for (int a = 0; a < dim; a++) cells *= std::floor((hi[a] - lo[a]) / h) + 1.0;
            if (cells <= 2.0 * (double)std::max<int64_t>(n, 1) + 64.0) break;
            if (doubling >= 2100 || !std::isfinite(h)) return SOPTX_E_INVALID_ARG;  // not a finite box
            h *= 2.0;
        }
        for (int a = 0; a < dim; a++) nc[a] = (int64_t)std::floor((hi[a] - lo[a]) / h) + 1;
        const int64_t ncell = nc[0] * nc[1] * nc[2];
        std::vector<int64_t> cell_ptr((size_t)ncell + 1, 0);
        std::vector<int64_t> cell_of((size_t)n);
        for (int64_t e = 0; e < n; e++) {
            int64_t ic[3] = {0, 0, 0};
            for (int a = 0; a < dim; a++)
                ic[a] = std::min<int64_t>(nc[a] - 1,
                                          std::max<int64_t>(0, (int64_t)std::floor((c[(size_t)e * dim + a] - lo[a]) / h)));
            cell_of[(size_t)e] = (ic[0] * nc[1] + ic[1]) * nc[2] + ic[2];
            cell_ptr[(size_t)cell_of[(size_t)e] + 1]++;
        }
        for (int64_t k = 0; k < ncell; k++) cell_ptr[(size_t)k + 1] += cell_ptr[(size_t)k];
        std::vector<int32_t> cell_el((size_t)n);
        {
            std::vector<int64_t> fill(cell_ptr.begin(), cell_ptr.end() - 1);
            for (int64_t e = 0; e < n; e++) cell_el[(size_t)fill[(size_t)cell_of[(size_t)e]]++] = (int32_t)e;
        }
        // rows in parallel chunks, concatenated in row order
        const int nth = (int)std::max<int64_t>(1, std::min<int64_t>(16, std::min<int64_t>(
                                                         (int64_t)std::thread::hardware_concurrency(), n / 4096 + 1)));
        std::vector<Rows> parts((size_t)nth);
        std::vector<int> failed((size_t)nth, 0);
        auto work = [&](int t) {
            const int64_t r0 = n * t / nth, r1 = n * (t + 1) / nth;
            try {
                search_rows(dim, c, rmin, lo, h, nc, cell_ptr, cell_el, r0, r1, parts[(size_t)t]);
            } catch (...) {
                failed[(size_t)t] = 1;
            }
        };
        std::vector<std::thread> th;
        for (int t = 1; t < nth; t++) {
            try {
                th.emplace_back(work, t);
            } catch (...) {
                work(t);  // no thread available: this one does the chunk
            }
        }
        work(0);
        for (auto &x : th) x.join();
        for (int f : failed)
            if (f) return SOPTX_E_OOM;
        int64_t nnz = 0;
        for (const auto &p : parts) nnz += (int64_t)p.col.size();
        if (nnz > INT32_MAX) return SOPTX_E_OVERFLOW;
        col.reserve((size_t)nnz);
        w.reserve((size_t)nnz);
        int64_t r = 0;
        for (const auto &p : parts) {
            for (int64_t k : p.cnt) {
                row_ptr[(size_t)r + 1] = row_ptr[(size_t)r] + (int32_t)k;
                r++;
            }
            col.insert(col.end(), p.col.begin(), p.col.end());
            w.insert(w.end(), p.w.begin(), p.w.end());
        }
        // row sums in ascending column order
        for (int64_t i = 0; i < n; i++) {
            double a = 0.0, b = 0.0;
            for (int32_t k = row_ptr[(size_t)i]; k < row_ptr[(size_t)i + 1]; k++) {
                a += w[(size_t)k] * v[(size_t)col[(size_t)k]];
                b += w[(size_t)k];
            }
            hsv[(size_t)i] = a;
            hs[(size_t)i] = b;
        }
    } catch (const std::bad_alloc &) {
        return SOPTX_E_OOM;
    }
    return SOPTX_OK;
}

}  // namespace

extern "C" {

int soptx_build_filter(const soptx_mesh *mesh, double rmin, soptx_filter *out, void *stream) {
    return soptx_build_filter_ex(mesh, rmin, 0, out, stream);
}

int soptx_build_filter_ex(const soptx_mesh *mesh, double rmin, int32_t flags, soptx_filter *out, void *stream) {
    if (!out) return SOPTX_E_INVALID_ARG;
    *out = nullptr;
    if (flags & ~SOPTX_FILTER_CSR_ONLY) return SOPTX_E_INVALID_ARG;
    HostFilter F;
    int rc = build_filter_host(mesh, rmin, F);
    if (rc) return rc;
    HostStencil T;
    bool stencil = false;
    try {
        stencil = !(flags & SOPTX_FILTER_CSR_ONLY) && detect_stencil(F, T);
    } catch (const std::bad_alloc &) {
        return SOPTX_E_OOM;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = F.n;

    soptx_filter_s *f = new (std::nothrow) soptx_filter_s();
    if (!f) return SOPTX_E_OOM;
    f->dim = mesh->dim;
    f->n = n;
    f->nnz = (int64_t)F.col.size();
    // rows per block of the product kernels: about kFilterChunk entries per
    // block (one LDS chunk) at the mean row length, within 1..256
    const double mean = n ? (double)f->nnz / (double)n : 1.0;
    f->rows_per_block = (int)std::max(1.0, std::min(256.0, std::floor((double)kFilterChunk / std::max(mean, 1.0))));
    if (hipGetDevice(&f->device) != hipSuccess) { free_filter(f); return SOPTX_E_DEVICE; }
    if ((rc = upload(f, F.row_ptr, &f->row_ptr, st)) || (rc = upload(f, F.col, &f->col, st)) ||
        (rc = upload(f, F.w, &f->w, st)) || (rc = upload(f, F.v, &f->v, st)) || (rc = upload(f, F.hsv, &f->hsv, st)) ||
        (rc = upload(f, F.hs, &f->hs, st))) {
        free_filter(f);
        return rc;
    }
    if (stencil) {
        f->S = (int)T.w.size();
        for (int k = 0; k < 3; k++) f->N[k] = T.N[k];
        if ((rc = upload(f, T.del, &f->sdel, st)) || (rc = upload(f, T.w, &f->sw, st))) {
            free_filter(f);
            return rc;
        }
    }
    if (hipStreamSynchronize(st) != hipSuccess) { free_filter(f); return SOPTX_E_DEVICE; }
    *out = f;
    return SOPTX_OK;
}

int soptx_filter_stencil_size(soptx_filter h, int32_t *S) {
    if (!h || !S) return SOPTX_E_INVALID_ARG;
    *S = h->S;
    return SOPTX_OK;
}

int soptx_filter_info(soptx_filter h, int64_t *n, int64_t *nnz, int32_t *rows_per_block) {
    if (!h || !n || !nnz) return SOPTX_E_INVALID_ARG;
    *n = h->n;
    *nnz = h->nnz;
    if (rows_per_block) *rows_per_block = h->rows_per_block;
    return SOPTX_OK;
}

int soptx_filter_copy(soptx_filter h, int32_t *h_row_ptr, int32_t *h_col, double *h_w, double *h_vol) {
    if (!h) return SOPTX_E_INVALID_ARG;
    DeviceGuard g(h->device);
    if (!g.ok) return SOPTX_E_DEVICE;
    hipError_t e = hipSuccess;
    if (h_row_ptr && h->row_ptr) e = hipMemcpy(h_row_ptr, h->row_ptr, (h->n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && h_col && h->col) e = hipMemcpy(h_col, h->col, h->nnz * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && h_w && h->w) e = hipMemcpy(h_w, h->w, h->nnz * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess && h_vol && h->v) e = hipMemcpy(h_vol, h->v, h->n * sizeof(double), hipMemcpyDeviceToHost);
    return finish(e);
}

int soptx_filter_sensitivity(soptx_filter h, const double *d_rho, const double *d_dc, double *d_dc_out,
                             void *stream) {
    if (!h) return SOPTX_E_INVALID_ARG;
    if (h->n == 0) return SOPTX_OK;
    if (!d_rho || !d_dc || !d_dc_out || d_dc_out == d_rho || d_dc_out == d_dc) return SOPTX_E_INVALID_ARG;
    DeviceGuard g(h->device);
    if (!g.ok) return SOPTX_E_DEVICE;
    return finish(launch_filter_sensitivity(args(h), h->rows_per_block, d_rho, d_dc, d_dc_out, static_cast<hipStream_t>(stream)));
}

int soptx_filter_density(soptx_filter h, const double *d_rho, double beta, double *d_rho_tilde, double *d_rho_bar,
                         void *stream) {
    if (!h) return SOPTX_E_INVALID_ARG;
    if (d_rho_bar && (!(beta >= 0.0) || !std::isfinite(beta))) return SOPTX_E_INVALID_ARG;
    if (h->n == 0) return SOPTX_OK;
    if (!d_rho || !d_rho_tilde || d_rho_tilde == d_rho || d_rho_bar == d_rho || d_rho_bar == d_rho_tilde)
        return SOPTX_E_INVALID_ARG;
    DeviceGuard g(h->device);
    if (!g.ok) return SOPTX_E_DEVICE;
    return finish(launch_filter_density(args(h), h->rows_per_block, d_rho, beta, d_rho_tilde, d_rho_bar,
                                        static_cast<hipStream_t>(stream)));
}

int soptx_filter_density_backward(soptx_filter h, const double *d_rho_tilde, double beta, const double *d_grad,
                                  double *d_grad_rho, void *stream) {
    if (!h) return SOPTX_E_INVALID_ARG;
    if (d_rho_tilde && (!(beta >= 0.0) || !std::isfinite(beta))) return SOPTX_E_INVALID_ARG;
    if (h->n == 0) return SOPTX_OK;
    if (!d_grad || !d_grad_rho || d_grad_rho == d_grad || d_grad_rho == d_rho_tilde) return SOPTX_E_INVALID_ARG;
    DeviceGuard g(h->device);
    if (!g.ok) return SOPTX_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *tmp = nullptr;
    int rc = get_workspace(h->device, st, (size_t)h->n, &tmp, 2);
    if (rc) return rc;
    return finish(launch_filter_backward(args(h), h->rows_per_block, d_rho_tilde, beta, d_grad, tmp, d_grad_rho, st));
}

int soptx_debug_filter_matrix(const soptx_mesh *mesh, double rmin, int64_t *n, int64_t *nnz, int32_t *row_ptr,
                              int32_t *col, double *w, double *vol, double *hsv, double *hs) {
    if (!n || !nnz) return SOPTX_E_INVALID_ARG;
    HostFilter F;
    int rc = build_filter_host(mesh, rmin, F);
    if (rc) return rc;
    *n = F.n;
    *nnz = (int64_t)F.col.size();
    if (row_ptr) std::copy(F.row_ptr.begin(), F.row_ptr.end(), row_ptr);
    if (col) std::copy(F.col.begin(), F.col.end(), col);
    if (w) std::copy(F.w.begin(), F.w.end(), w);
    if (vol) std::copy(F.v.begin(), F.v.end(), vol);
    if (hsv) std::copy(F.hsv.begin(), F.hsv.end(), hsv);
    if (hs) std::copy(F.hs.begin(), F.hs.end(), hs);
    return SOPTX_OK;
}

int soptx_debug_filter_stencil(const soptx_mesh *mesh, double rmin, int32_t *S, int64_t *N) {
    if (!S || !N) return SOPTX_E_INVALID_ARG;
    HostFilter F;
    int rc = build_filter_host(mesh, rmin, F);
    if (rc) return rc;
    HostStencil T;
    try {
        *S = detect_stencil(F, T) ? (int32_t)T.w.size() : 0;
    } catch (const std::bad_alloc &) {
        return SOPTX_E_OOM;
    }
    for (int k = 0; k < 3; k++) N[k] = *S ? T.N[k] : 0;
    return SOPTX_OK;
}

void soptx_destroy_filter(soptx_filter h) {
    if (!h) return;
    DeviceGuard g(h->device);
    free_filter(h);
}

}  // extern "C"
