// Element-independent reference data (the invariant part of "fast assembly",
// Sec. 3.2.2 and Sec. 5.5): basis gradients on the reference element, the
// reference tensor M[i][j][m][n] = int_ref d_m phi_i d_n phi_j, and the exact
// quadrature rules used by the element-energy kernel.
//
// The "symbolic" variant integrates M exactly in rational arithmetic (the
// analogue of the paper's SymPy precomputation); the "quadrature" variant uses
// the element's exact FP64 rule.
#include "internal.h"

#include <cmath>
#include <cstdint>
#include <map>
#include <numeric>
#include <vector>

namespace soptx {

// ----------------------------------------------------------- exact rationals
namespace {

struct Rat {
    int64_t n = 0, d = 1;
    Rat() = default;
    Rat(int64_t a, int64_t b = 1) : n(a), d(b) { norm(); }
    void norm() {
        if (d < 0) { n = -n; d = -d; }
        int64_t g = std::gcd(n < 0 ? -n : n, d);
        if (g > 1) { n /= g; d /= g; }
        if (n == 0) d = 1;
    }
};
Rat operator+(Rat a, Rat b) { return Rat(a.n * b.d + b.n * a.d, a.d * b.d); }
Rat operator*(Rat a, Rat b) { return Rat(a.n * b.n, a.d * b.d); }

// polynomial in up to 3 variables: exponent triple -> coefficient
using Mono = std::array<int, 3>;
using Poly = std::map<Mono, Rat>;

Poly padd(const Poly &a, const Poly &b) {
    Poly r = a;
    for (auto &kv : b) {
        Rat s = r[kv.first] + kv.second;
        if (s.n == 0) r.erase(kv.first); else r[kv.first] = s;
    }
    return r;
}
Poly pmul(const Poly &a, const Poly &b) {
    Poly r;
    for (auto &x : a)
        for (auto &y : b) {
            Mono m{x.first[0] + y.first[0], x.first[1] + y.first[1], x.first[2] + y.first[2]};
            Rat s = r[m] + x.second * y.second;
            if (s.n == 0) r.erase(m); else r[m] = s;
        }
    return r;
}
Poly pscale(const Poly &a, Rat c) {
    Poly r;
    if (c.n == 0) return r;
    for (auto &x : a) r[x.first] = x.second * c;
    return r;
}
Poly pdiff(const Poly &a, int v) {
    Poly r;
    for (auto &x : a) {
        if (x.first[v] == 0) continue;
        Mono m = x.first;
        Rat c = x.second * Rat(m[v]);
        m[v] -= 1;
        r[m] = c;
    }
    return r;
}
Poly pconst(int64_t c) { Poly r; if (c) r[Mono{0, 0, 0}] = Rat(c); return r; }
Poly pvar(int v) { Poly r; Mono m{0, 0, 0}; m[v] = 1; r[m] = Rat(1); return r; }

int64_t fact(int k) { int64_t f = 1; for (int i = 2; i <= k; i++) f *= i; return f; }

// exact integral over the reference cube [0,1]^dim or unit simplex
Rat integrate(const Poly &p, int dim, bool simplex) {
    Rat s(0);
    for (auto &x : p) {
        Rat v(1);
        if (simplex) {
            int64_t num = 1;
            int tot = 0;
            for (int k = 0; k < dim; k++) { num *= fact(x.first[k]); tot += x.first[k]; }
            v = Rat(num, fact(tot + dim));
        } else {
            for (int k = 0; k < dim; k++) v = v * Rat(1, x.first[k] + 1);
        }
        s = s + x.second * v;
    }
    return s;
}

// reference basis functions as exact polynomials
std::vector<Poly> basis_polys(int elem) {
    std::vector<Poly> ph;
    auto one_minus = [](int v) { return padd(pconst(1), pscale(pvar(v), Rat(-1))); };
    if (elem == SOPTX_QUAD4 || elem == SOPTX_HEX8) {
        const int dim = elem == SOPTX_QUAD4 ? 2 : 3;
        const int n = elem == SOPTX_QUAD4 ? 4 : 8;
        for (int i = 0; i < n; i++) {
            Poly p = pconst(1);
            for (int a = 0; a < dim; a++) {
                int bit = corner_bit(elem, i, a);
                p = pmul(p, bit ? pvar(a) : one_minus(a));
            }
            ph.push_back(p);
        }
    } else if (elem == SOPTX_HEX27) {
        // 1D quadratic Lagrange on {0, 1/2, 1}: (1-t)(1-2t), 4t(1-t), t(2t-1)
        auto lag = [&](int k, int v) {
            Poly t = pvar(v);
            if (k == 0) return pmul(one_minus(v), padd(pconst(1), pscale(t, Rat(-2))));
            if (k == 1) return pscale(pmul(t, one_minus(v)), Rat(4));
            return pmul(t, padd(pscale(t, Rat(2)), pconst(-1)));
        };
        for (int i = 0; i < 27; i++) {
            Poly p = pconst(1);
            for (int a = 0; a < 3; a++) p = pmul(p, lag(lattice_index(i, a), a));
            ph.push_back(p);
        }
    } else if (elem == SOPTX_TRI3) {
        ph.push_back(padd(pconst(1), padd(pscale(pvar(0), Rat(-1)), pscale(pvar(1), Rat(-1)))));
        ph.push_back(pvar(0));
        ph.push_back(pvar(1));
    } else if (elem == SOPTX_TET10) {
        Poly L[4];
        L[0] = padd(pconst(1), padd(pscale(pvar(0), Rat(-1)),
                                    padd(pscale(pvar(1), Rat(-1)), pscale(pvar(2), Rat(-1)))));
        L[1] = pvar(0); L[2] = pvar(1); L[3] = pvar(2);
        for (int i = 0; i < 4; i++)
            ph.push_back(pmul(L[i], padd(pscale(L[i], Rat(2)), pconst(-1))));
        static const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
        for (int k = 0; k < 6; k++) ph.push_back(pscale(pmul(L[E[k][0]], L[E[k][1]]), Rat(4)));
    }
    return ph;
}

}  // namespace

// corner (0/1) of node i of a Q1 element along axis a (Q2 hexahedra: the
// same for their corner nodes 0-7)
int corner_bit(int elem, int i, int a) {
    static const int Q[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
    static const int H[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                                {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};
    return elem == SOPTX_QUAD4 ? Q[i][a] : H[i][a];
}

// lattice index (0, 1, 2: reference coordinate 0, 1/2, 1) of node i of the Q2
// hexahedron along axis a: corners 0-7 as for Q1, then the other 19 lattice
// points in ascending a + 3b + 9c
int lattice_index(int i, int a) {
    struct Table { int v[27][3]; };
    static const Table L = [] {  // built once, thread-safe
        Table t{};
        for (int k = 0; k < 8; k++)
            for (int m = 0; m < 3; m++) t.v[k][m] = 2 * corner_bit(SOPTX_HEX8, k, m);
        int n = 8;
        for (int z = 0; z < 3; z++)
            for (int y = 0; y < 3; y++)
                for (int x = 0; x < 3; x++)
                    if (x == 1 || y == 1 || z == 1) { t.v[n][0] = x; t.v[n][1] = y; t.v[n][2] = z; n++; }
        return t;
    }();
    return L.v[i][a];
}

// ----------------------------------------------------------- quadrature rules
// Gauss 2-point per axis on [0,1] for Q1 (exact to degree 3 per variable),
// 3-point for Q2 hexahedra (1/2 -+ sqrt(3/5)/2 and 1/2, weights 5/18, 8/18,
// 5/18: exact to degree 5 per variable);
// centroid rule for P1 (gradients are constant); the symmetric 4-point rule of
// degree 2 for P2 tetrahedra (barycentric (a,b,b,b), a = (5+3 sqrt5)/20,
// b = (5-sqrt5)/20, weight 1/24 each).
void quadrature_rule(int elem, std::vector<double> &pts, std::vector<double> &wts) {
    pts.clear();
    wts.clear();
    const double g0 = 0.5 - 0.5 / std::sqrt(3.0), g1 = 0.5 + 0.5 / std::sqrt(3.0);
    const double g[2] = {g0, g1};
    switch (elem) {
    case SOPTX_QUAD4:
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) { pts.push_back(g[a]); pts.push_back(g[b]); wts.push_back(0.25); }
        break;
    case SOPTX_HEX8:
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++)
                for (int c = 0; c < 2; c++) {
                    pts.push_back(g[a]); pts.push_back(g[b]); pts.push_back(g[c]);
                    wts.push_back(0.125);
                }
        break;
    case SOPTX_HEX27: {
        const double h[3] = {0.5 - 0.5 * std::sqrt(0.6), 0.5, 0.5 + 0.5 * std::sqrt(0.6)};
        const double w[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++)
                for (int c = 0; c < 3; c++) {
                    pts.push_back(h[a]); pts.push_back(h[b]); pts.push_back(h[c]);
                    wts.push_back(w[a] * w[b] * w[c]);
                }
        break;
    }
    case SOPTX_TRI3:
        pts.push_back(1.0 / 3.0); pts.push_back(1.0 / 3.0); wts.push_back(0.5);
        break;
    case SOPTX_TET10: {
        const double a = (5.0 + 3.0 * std::sqrt(5.0)) / 20.0, b = (5.0 - std::sqrt(5.0)) / 20.0;
        const double bary[4][3] = {{b, b, b}, {a, b, b}, {b, a, b}, {b, b, a}};
        for (int q = 0; q < 4; q++) {
            for (int k = 0; k < 3; k++) pts.push_back(bary[q][k]);
            wts.push_back(1.0 / 24.0);
        }
        break;
    }
    default:
        break;
    }
}

// gradients d phi_i / d xi_m at xi, evaluated from the exact polynomials
static void eval_grads(const std::vector<Poly> &ph, int dim, const double *xi, double *out) {
    for (size_t i = 0; i < ph.size(); i++)
        for (int m = 0; m < dim; m++) {
            Poly d = pdiff(ph[i], m);
            double s = 0.0;
            for (auto &x : d) {
                double t = double(x.second.n) / double(x.second.d);
                for (int k = 0; k < dim; k++) t *= std::pow(xi[k], x.first[k]);
                s += t;
            }
            out[i * dim + m] = s;
        }
}

int reference_tensor(int elem, int method, double *M) {
    const int dim = elem_dim(elem), nen = elem_nen(elem);
    if (dim < 0) return SOPTX_E_UNSUPPORTED_ELEM;
    std::vector<Poly> ph = basis_polys(elem);
    const bool simplex = (elem == SOPTX_TRI3 || elem == SOPTX_TET10);
    if (method == SOPTX_REF_SYMBOLIC) {
        std::vector<Poly> g(nen * dim);
        for (int i = 0; i < nen; i++)
            for (int m = 0; m < dim; m++) g[i * dim + m] = pdiff(ph[i], m);
        for (int i = 0; i < nen; i++)
            for (int j = 0; j < nen; j++)
                for (int m = 0; m < dim; m++)
                    for (int n = 0; n < dim; n++) {
                        Rat r = integrate(pmul(g[i * dim + m], g[j * dim + n]), dim, simplex);
                        M[((i * nen + j) * dim + m) * dim + n] = double(r.n) / double(r.d);
                    }
        return SOPTX_OK;
    }
    if (method == SOPTX_REF_QUADRATURE) {
        std::vector<double> pts, wts;
        quadrature_rule(elem, pts, wts);
        std::vector<double> gq(nen * dim);
        for (int k = 0; k < nen * nen * dim * dim; k++) M[k] = 0.0;
        for (size_t q = 0; q < wts.size(); q++) {
            eval_grads(ph, dim, &pts[q * dim], gq.data());
            for (int i = 0; i < nen; i++)
                for (int j = 0; j < nen; j++)
                    for (int m = 0; m < dim; m++)
                        for (int n = 0; n < dim; n++)
                            M[((i * nen + j) * dim + m) * dim + n] += wts[q] * gq[i * dim + m] * gq[j * dim + n];
        }
        return SOPTX_OK;
    }
    return SOPTX_E_INVALID_ARG;
}

int reference_qp_grads(int elem, std::vector<double> &wts, std::vector<double> &grads) {
    const int dim = elem_dim(elem), nen = elem_nen(elem);
    if (dim < 0) return SOPTX_E_UNSUPPORTED_ELEM;
    std::vector<double> pts;
    quadrature_rule(elem, pts, wts);
    std::vector<Poly> ph = basis_polys(elem);
    grads.assign(wts.size() * nen * dim, 0.0);
    for (size_t q = 0; q < wts.size(); q++) eval_grads(ph, dim, &pts[q * dim], &grads[q * nen * dim]);
    return SOPTX_OK;
}

}  // namespace soptx
