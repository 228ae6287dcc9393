/*
 * oracle.c -- plain, slow, FP64 CPU reference for SIMP stiffness assembly,
 * compliance and compliance sensitivity.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the HIP library.
 *
 * What it computes (paper, Section 2.2 "Compliance Minimization Problem" and
 * Eq. (cmpd); Section 2.1 for the modified SIMP law; Appendix D for the
 * element sensitivity):
 *
 *   E(rho)      = Emin + rho^p (E0 - Emin)                  (Sec. 2.1)
 *   K(rho)      = sum_e E(rho_e) K_e^0, K_e^0 at unit E     (Eq. cmpd)
 *   c           = F^T U = U^T K U (twice the strain energy) (Eq. cmpc/cmpd)
 *   dc/drho_e   = -p rho_e^(p-1) (E0 - Emin) u_e^T K_e^0 u_e  (App. D: the
 *                 derivative of -E(rho_e) u_e^T ke0 u_e at fixed u)
 *
 * K_e^0 is built the "standard" way (the baseline of Sec. 5.5 / Table 1):
 * numerical quadrature of B^T D B |det J| at each quadrature point, with J
 * re-evaluated at every point (no affine shortcut, no separated reference
 * tensor).  Quadrature rules are exact for affine elements:
 *   Q1 quad 2x2 Gauss, Q1 hex 2x2x2 Gauss, P1 tri 1-point centroid,
 *   P2 tet 4-point degree-2 rule (a=(5+3 sqrt5)/20, b=(5-sqrt5)/20),
 *   Q2 hex 3x3x3 Gauss (exact to degree 5 in each variable).
 *
 * The Q2 hexahedron (27-node triquadratic Lagrange element) is a variant
 * beyond the paper's examples, which use linear elements (Sec. 3.2.2); the
 * underlying platform offers elements of any order (Sec. 1).  Node order:
 * the 8 corners as for Q1, then the other 19 points of the 3x3x3 lattice
 * {0, 1/2, 1}^3 in ascending a + 3b + 9c, with (a, b, c) the lattice indices
 * along x, y, z.
 *
 * Elasticity matrix D (Sec. 3.2.1 material module; Sec. 4.2 uses plane
 * stress with E=1, nu=0.3): Voigt notation with engineering shear strains.
 *
 * Sparse pattern: the set {(dof(e,i), dof(e,j))}, rows ascending, columns
 * ascending and unique within a row, structural zeros kept.
 * Summation order of every stored value: elements in ascending id, then the
 * local row, then the local column (the order of the element loop below).
 *
 * Dirichlet conditions (zero prescribed values, Appendices A-C): every fixed
 * dof r gets K[r,:] = 0, K[:,r] = 0, K[r,r] = 1; the pattern is unchanged.
 *
 * All functions return 0 on success and a negative value on bad input.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { E_QUAD4 = 1, E_TRI3 = 2, E_HEX8 = 3, E_TET10 = 4, E_HEX27 = 5 };

#define MAXNEN 27
#define MAXLDOF 81
#define MAXQ 27

static int elem_dim(int elem) {
    switch (elem) {
    case E_QUAD4: case E_TRI3: return 2;
    case E_HEX8: case E_TET10: case E_HEX27: return 3;
    default: return -1;
    }
}

static int elem_nen(int elem) {
    switch (elem) {
    case E_QUAD4: return 4;
    case E_TRI3: return 3;
    case E_HEX8: return 8;
    case E_TET10: return 10;
    case E_HEX27: return 27;
    default: return -1;
    }
}

int oracle_elem_dim(int elem) { return elem_dim(elem); }
int oracle_elem_nen(int elem) { return elem_nen(elem); }

/* ----------------------------------------------------------------------
 * Reference elements and shape functions.
 *   Q1: reference [0,1]^d, tensor-product linear Lagrange functions.
 *   P1: reference simplex with vertices 0, e1, e2; barycentric functions.
 *   P2: reference simplex 0,e1,e2,e3; vertex functions L(2L-1),
 *       edge functions 4 La Lb for edges 01,02,03,12,13,23.
 * dphi[i*dim + m] = d phi_i / d xi_m.
 * ---------------------------------------------------------------------- */
static const int QUAD_CORNER[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
static const int HEX_CORNER[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                                     {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};
static const int TET_EDGE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

/* 1D linear Lagrange function on [0,1] for corner bit c, and its derivative */
static double lin(int c, double t) { return c ? t : 1.0 - t; }
static double dlin(int c) { return c ? 1.0 : -1.0; }

/* 1D quadratic Lagrange functions on [0,1] with nodes 0, 1/2, 1 (index k):
 * l0 = (1-t)(1-2t), l1 = 4t(1-t), l2 = t(2t-1), and their derivatives */
static double quad1(int k, double t) {
    return k == 0 ? (1.0 - t) * (1.0 - 2.0 * t) : k == 1 ? 4.0 * t * (1.0 - t) : t * (2.0 * t - 1.0);
}
static double dquad1(int k, double t) { return k == 0 ? 4.0 * t - 3.0 : k == 1 ? 4.0 - 8.0 * t : 4.0 * t - 1.0; }

/* lattice indices (a, b, c) of the Q2 hexahedron's node i, in the order
 * stated at the top of this file */
static void hex27_node(int i, int *abc) {
    int n = 8, a, b, c;
    if (i < 8) {
        abc[0] = 2 * HEX_CORNER[i][0]; abc[1] = 2 * HEX_CORNER[i][1]; abc[2] = 2 * HEX_CORNER[i][2];
        return;
    }
    for (c = 0; c < 3; c++)
        for (b = 0; b < 3; b++)
            for (a = 0; a < 3; a++) {
                if (a != 1 && b != 1 && c != 1) continue; /* a corner */
                if (n == i) { abc[0] = a; abc[1] = b; abc[2] = c; return; }
                n++;
            }
}
int oracle_hex27_node(int i, int *abc) {
    if (i < 0 || i >= 27) return -1;
    hex27_node(i, abc);
    return 0;
}

int oracle_ref_basis(int elem, const double *xi, double *phi, double *dphi) {
    int i;
    switch (elem) {
    case E_QUAD4:
        for (i = 0; i < 4; i++) {
            int cx = QUAD_CORNER[i][0], cy = QUAD_CORNER[i][1];
            phi[i] = lin(cx, xi[0]) * lin(cy, xi[1]);
            dphi[2 * i + 0] = dlin(cx) * lin(cy, xi[1]);
            dphi[2 * i + 1] = lin(cx, xi[0]) * dlin(cy);
        }
        return 0;
    case E_HEX8:
        for (i = 0; i < 8; i++) {
            int cx = HEX_CORNER[i][0], cy = HEX_CORNER[i][1], cz = HEX_CORNER[i][2];
            phi[i] = lin(cx, xi[0]) * lin(cy, xi[1]) * lin(cz, xi[2]);
            dphi[3 * i + 0] = dlin(cx) * lin(cy, xi[1]) * lin(cz, xi[2]);
            dphi[3 * i + 1] = lin(cx, xi[0]) * dlin(cy) * lin(cz, xi[2]);
            dphi[3 * i + 2] = lin(cx, xi[0]) * lin(cy, xi[1]) * dlin(cz);
        }
        return 0;
    case E_HEX27:
        for (i = 0; i < 27; i++) {
            int k[3];
            hex27_node(i, k);
            phi[i] = quad1(k[0], xi[0]) * quad1(k[1], xi[1]) * quad1(k[2], xi[2]);
            dphi[3 * i + 0] = dquad1(k[0], xi[0]) * quad1(k[1], xi[1]) * quad1(k[2], xi[2]);
            dphi[3 * i + 1] = quad1(k[0], xi[0]) * dquad1(k[1], xi[1]) * quad1(k[2], xi[2]);
            dphi[3 * i + 2] = quad1(k[0], xi[0]) * quad1(k[1], xi[1]) * dquad1(k[2], xi[2]);
        }
        return 0;
    case E_TRI3:
        phi[0] = 1.0 - xi[0] - xi[1];
        phi[1] = xi[0];
        phi[2] = xi[1];
        dphi[0] = -1.0; dphi[1] = -1.0;
        dphi[2] = 1.0;  dphi[3] = 0.0;
        dphi[4] = 0.0;  dphi[5] = 1.0;
        return 0;
    case E_TET10: {
        /* barycentric coordinates and their constant gradients */
        double L[4] = {1.0 - xi[0] - xi[1] - xi[2], xi[0], xi[1], xi[2]};
        double dL[4][3] = {{-1, -1, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        int m;
        for (i = 0; i < 4; i++) {
            phi[i] = L[i] * (2.0 * L[i] - 1.0);
            for (m = 0; m < 3; m++) dphi[3 * i + m] = (4.0 * L[i] - 1.0) * dL[i][m];
        }
        for (i = 0; i < 6; i++) {
            int a = TET_EDGE[i][0], b = TET_EDGE[i][1];
            phi[4 + i] = 4.0 * L[a] * L[b];
            for (m = 0; m < 3; m++)
                dphi[3 * (4 + i) + m] = 4.0 * (dL[a][m] * L[b] + L[a] * dL[b][m]);
        }
        return 0;
    }
    default:
        return -1;
    }
}

/* Quadrature rules on the reference elements (weights sum to the reference measure). */
int oracle_quadrature(int elem, int *nq, double *pts, double *wts) {
    int q;
    switch (elem) {
    case E_QUAD4: {
        double g[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
        int a, b;
        q = 0;
        for (a = 0; a < 2; a++)
            for (b = 0; b < 2; b++) {
                pts[2 * q] = g[a]; pts[2 * q + 1] = g[b]; wts[q] = 0.25; q++;
            }
        *nq = 4;
        return 0;
    }
    case E_HEX8: {
        double g[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
        int a, b, c;
        q = 0;
        for (a = 0; a < 2; a++)
            for (b = 0; b < 2; b++)
                for (c = 0; c < 2; c++) {
                    pts[3 * q] = g[a]; pts[3 * q + 1] = g[b]; pts[3 * q + 2] = g[c];
                    wts[q] = 0.125; q++;
                }
        *nq = 8;
        return 0;
    }
    case E_HEX27: {
        /* 3-point Gauss-Legendre on [0,1]: 1/2 -+ sqrt(3/5)/2 and 1/2,
         * weights 5/18, 8/18, 5/18 */
        double g[3] = {0.5 - 0.5 * sqrt(0.6), 0.5, 0.5 + 0.5 * sqrt(0.6)};
        double w[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
        int a, b, c;
        q = 0;
        for (a = 0; a < 3; a++)
            for (b = 0; b < 3; b++)
                for (c = 0; c < 3; c++) {
                    pts[3 * q] = g[a]; pts[3 * q + 1] = g[b]; pts[3 * q + 2] = g[c];
                    wts[q] = w[a] * w[b] * w[c]; q++;
                }
        *nq = 27;
        return 0;
    }
    case E_TRI3:
        pts[0] = 1.0 / 3.0; pts[1] = 1.0 / 3.0; wts[0] = 0.5;
        *nq = 1;
        return 0;
    case E_TET10: {
        double a = (5.0 + 3.0 * sqrt(5.0)) / 20.0, b = (5.0 - sqrt(5.0)) / 20.0;
        /* barycentric (a,b,b,b) and permutations; xi = (L1, L2, L3) */
        double bary[4][4] = {{a, b, b, b}, {b, a, b, b}, {b, b, a, b}, {b, b, b, a}};
        for (q = 0; q < 4; q++) {
            pts[3 * q + 0] = bary[q][1];
            pts[3 * q + 1] = bary[q][2];
            pts[3 * q + 2] = bary[q][3];
            wts[q] = 1.0 / 24.0;
        }
        *nq = 4;
        return 0;
    }
    default:
        return -1;
    }
}

/* Elasticity matrix in Voigt notation with engineering shear strains.
 * 2D: (exx, eyy, gxy); plane stress unless plane_strain != 0.
 * 3D: (exx, eyy, ezz, gyz, gxz, gxy), Lame constants
 *     lambda = E nu / ((1+nu)(1-2nu)), mu = E / (2(1+nu)). */
int oracle_D(int dim, int plane_strain, double E, double nu, double *D) {
    int k;
    if (dim == 2) {
        for (k = 0; k < 9; k++) D[k] = 0.0;
        if (!plane_strain) {
            double c = E / (1.0 - nu * nu);
            D[0] = c; D[1] = c * nu;
            D[3] = c * nu; D[4] = c;
            D[8] = c * (1.0 - nu) / 2.0;
        } else {
            double c = E / ((1.0 + nu) * (1.0 - 2.0 * nu));
            D[0] = c * (1.0 - nu); D[1] = c * nu;
            D[3] = c * nu; D[4] = c * (1.0 - nu);
            D[8] = c * (1.0 - 2.0 * nu) / 2.0;
        }
        return 0;
    }
    if (dim == 3) {
        double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
        double mu = E / (2.0 * (1.0 + nu));
        int a, b;
        for (k = 0; k < 36; k++) D[k] = 0.0;
        for (a = 0; a < 3; a++)
            for (b = 0; b < 3; b++) D[6 * a + b] = lam + (a == b ? 2.0 * mu : 0.0);
        for (a = 3; a < 6; a++) D[6 * a + a] = mu;
        return 0;
    }
    return -1;
}

/* Determinant and inverse of a dim x dim matrix (row-major). */
static double det_inv(int dim, const double *J, double *Ji) {
    double d;
    if (dim == 2) {
        d = J[0] * J[3] - J[1] * J[2];
        Ji[0] = J[3] / d; Ji[1] = -J[1] / d;
        Ji[2] = -J[2] / d; Ji[3] = J[0] / d;
        return d;
    }
    d = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
        J[2] * (J[3] * J[7] - J[4] * J[6]);
    Ji[0] = (J[4] * J[8] - J[5] * J[7]) / d;
    Ji[1] = (J[2] * J[7] - J[1] * J[8]) / d;
    Ji[2] = (J[1] * J[5] - J[2] * J[4]) / d;
    Ji[3] = (J[5] * J[6] - J[3] * J[8]) / d;
    Ji[4] = (J[0] * J[8] - J[2] * J[6]) / d;
    Ji[5] = (J[2] * J[3] - J[0] * J[5]) / d;
    Ji[6] = (J[3] * J[7] - J[4] * J[6]) / d;
    Ji[7] = (J[1] * J[6] - J[0] * J[7]) / d;
    Ji[8] = (J[0] * J[4] - J[1] * J[3]) / d;
    return d;
}

/* Strain-displacement matrix B (nstrain x ldof) from physical gradients g[i*dim+a]. */
static void build_B(int dim, int nen, const double *g, double *B) {
    int ldof = dim * nen, i;
    if (dim == 2) {
        memset(B, 0, sizeof(double) * 3 * ldof);
        for (i = 0; i < nen; i++) {
            double gx = g[2 * i], gy = g[2 * i + 1];
            B[0 * ldof + 2 * i + 0] = gx;
            B[1 * ldof + 2 * i + 1] = gy;
            B[2 * ldof + 2 * i + 0] = gy;
            B[2 * ldof + 2 * i + 1] = gx;
        }
    } else {
        memset(B, 0, sizeof(double) * 6 * ldof);
        for (i = 0; i < nen; i++) {
            double gx = g[3 * i], gy = g[3 * i + 1], gz = g[3 * i + 2];
            B[0 * ldof + 3 * i + 0] = gx;
            B[1 * ldof + 3 * i + 1] = gy;
            B[2 * ldof + 3 * i + 2] = gz;
            B[3 * ldof + 3 * i + 1] = gz; B[3 * ldof + 3 * i + 2] = gy;
            B[4 * ldof + 3 * i + 0] = gz; B[4 * ldof + 3 * i + 2] = gx;
            B[5 * ldof + 3 * i + 0] = gy; B[5 * ldof + 3 * i + 1] = gx;
        }
    }
}

/* Element stiffness at unit Young's modulus (K_e^0 of Eq. cmpd), standard
 * quadrature: Ke = sum_q w_q |det J(xi_q)| B(xi_q)^T D B(xi_q).
 * xe: node coordinates of the element [nen][dim]; Ke: [ldof][ldof].
 * Returns the (signed) determinant at the first quadrature point, or 0 on error. */
double oracle_element_ke0(int elem, const double *xe, double nu, int plane_strain, double *Ke) {
    int dim = elem_dim(elem), nen = elem_nen(elem);
    int ldof, nq, q, i, j, a, b, m, ns;
    double pts[3 * MAXQ], wts[MAXQ], D[36], phi[MAXNEN], dphi[3 * MAXNEN];
    double B[6 * MAXLDOF], DB[6 * MAXLDOF], g[3 * MAXNEN], J[9], Ji[9], det, det0 = 0.0;
    if (dim < 0) return 0.0;
    ldof = dim * nen;
    ns = dim == 2 ? 3 : 6;
    oracle_quadrature(elem, &nq, pts, wts);
    oracle_D(dim, plane_strain, 1.0, nu, D);
    memset(Ke, 0, sizeof(double) * ldof * ldof);
    for (q = 0; q < nq; q++) {
        oracle_ref_basis(elem, pts + dim * q, phi, dphi);
        /* J[a][m] = d x_a / d xi_m = sum_i x_{i,a} dphi_i/dxi_m */
        for (a = 0; a < dim; a++)
            for (m = 0; m < dim; m++) {
                double s = 0.0;
                for (i = 0; i < nen; i++) s += xe[dim * i + a] * dphi[dim * i + m];
                J[dim * a + m] = s;
            }
        det = det_inv(dim, J, Ji);
        if (q == 0) det0 = det;
        /* physical gradient: d phi_i/dx_a = sum_m dphi_i/dxi_m * (J^-1)[m][a] */
        for (i = 0; i < nen; i++)
            for (a = 0; a < dim; a++) {
                double s = 0.0;
                for (m = 0; m < dim; m++) s += dphi[dim * i + m] * Ji[dim * m + a];
                g[dim * i + a] = s;
            }
        build_B(dim, nen, g, B);
        for (a = 0; a < ns; a++)
            for (j = 0; j < ldof; j++) {
                double s = 0.0;
                for (b = 0; b < ns; b++) s += D[ns * a + b] * B[ldof * b + j];
                DB[ldof * a + j] = s;
            }
        for (i = 0; i < ldof; i++)
            for (j = 0; j < ldof; j++) {
                double s = 0.0;
                for (a = 0; a < ns; a++) s += B[ldof * a + i] * DB[ldof * a + j];
                Ke[ldof * i + j] += wts[q] * fabs(det) * s;
            }
    }
    return det0;
}

/* ------------------------------------------------------------ pattern */

static int cmp_i64(const void *x, const void *y) {
    int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    return (a > b) - (a < b);
}

/* Node-pair set {(cells[e][i], cells[e][j])}, sorted and unique, as keys
 * I*n_nodes+J.  keys must hold n_cells*nen*nen entries.  Returns the count. */
int64_t oracle_node_pairs(int elem, int64_t n_nodes, int64_t n_cells, const int32_t *cells,
                          int64_t *keys) {
    int nen = elem_nen(elem);
    int64_t e, n = 0, k, u;
    int i, j;
    if (nen < 0) return -1;
    for (e = 0; e < n_cells; e++)
        for (i = 0; i < nen; i++)
            for (j = 0; j < nen; j++)
                keys[n++] = (int64_t)cells[e * nen + i] * n_nodes + cells[e * nen + j];
    qsort(keys, (size_t)n, sizeof(int64_t), cmp_i64);
    u = 0;
    for (k = 0; k < n; k++)
        if (u == 0 || keys[k] != keys[u - 1]) keys[u++] = keys[k];
    return u;
}

/* CSR of the dof pattern from the unique node pairs.  Because every local dof
 * pair (i,a),(j,b) of an element appears, the dof set is exactly
 * {(dim*I+a, dim*J+b) : (I,J) a node pair, 0<=a,b<dim}; row dim*I+a lists
 * dim*J+b for the neighbours J of I in ascending order, then b ascending.
 * row_ptr: [ndof+1]; col_idx: [npairs*dim*dim]. */
int oracle_pattern_from_pairs(int dim, int64_t n_nodes, int64_t npairs, const int64_t *keys,
                              int64_t *row_ptr, int32_t *col_idx) {
    int64_t ndof = dim * n_nodes, k = 0, I, pos = 0;
    int a, b;
    row_ptr[0] = 0;
    for (I = 0; I < n_nodes; I++) {
        int64_t k0 = k, k1;
        while (k < npairs && keys[k] / n_nodes == I) k++;
        k1 = k;
        for (a = 0; a < dim; a++) {
            int64_t kk;
            for (kk = k0; kk < k1; kk++) {
                int64_t J = keys[kk] % n_nodes;
                for (b = 0; b < dim; b++) col_idx[pos++] = (int32_t)(dim * J + b);
            }
            row_ptr[dim * I + a + 1] = pos;
        }
    }
    (void)ndof;
    return 0;
}

/* position of column c in row r (binary search), -1 if absent */
static int64_t find_slot(const int64_t *row_ptr, const int32_t *col_idx, int64_t r, int32_t c) {
    int64_t lo = row_ptr[r], hi = row_ptr[r + 1] - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col_idx[mid] == c) return mid;
        if (col_idx[mid] < c) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

static void gather_coords(int dim, int nen, const double *coords, const int32_t *cell, double *xe) {
    int i, a;
    for (i = 0; i < nen; i++)
        for (a = 0; a < dim; a++) xe[dim * i + a] = coords[(int64_t)cell[i] * dim + a];
}

/* Modified SIMP law of Sec. 2.1 and its derivative. */
static double simp_E(double rho, double E0, double Emin, double p) {
    return Emin + pow(rho, p) * (E0 - Emin);
}
static double simp_dE(double rho, double E0, double Emin, double p) {
    return p * pow(rho, p - 1.0) * (E0 - Emin);
}

/* K_vals = sum_e E(rho_e) K_e^0 scattered into the pattern, elements in
 * ascending order (Eq. cmpd), then the Dirichlet rows/columns if mask != NULL.
 * Returns 0, or -2 if an element entry has no slot in the pattern. */
int oracle_assemble(int elem, int64_t n_nodes, const double *coords, int64_t n_cells,
                    const int32_t *cells, const double *rho, double E0, double Emin, double p,
                    double nu, int plane_strain, const uint8_t *mask, const int64_t *row_ptr,
                    const int32_t *col_idx, double *K) {
    int dim = elem_dim(elem), nen = elem_nen(elem), ldof, i, j;
    int64_t e, ndof, r, k;
    double xe[3 * MAXNEN], Ke[MAXLDOF * MAXLDOF];
    if (dim < 0) return -1;
    ldof = dim * nen;
    ndof = dim * n_nodes;
    memset(K, 0, sizeof(double) * row_ptr[ndof]);
    for (e = 0; e < n_cells; e++) {
        const int32_t *cell = cells + e * nen;
        double Ee = simp_E(rho[e], E0, Emin, p);
        gather_coords(dim, nen, coords, cell, xe);
        oracle_element_ke0(elem, xe, nu, plane_strain, Ke);
        for (i = 0; i < ldof; i++) {
            int64_t gr = (int64_t)dim * cell[i / dim] + i % dim;
            for (j = 0; j < ldof; j++) {
                int32_t gc = (int32_t)(dim * cell[j / dim] + j % dim);
                int64_t s = find_slot(row_ptr, col_idx, gr, gc);
                if (s < 0) return -2;
                K[s] += Ee * Ke[ldof * i + j];
            }
        }
    }
    if (mask) {
        for (r = 0; r < ndof; r++)
            for (k = row_ptr[r]; k < row_ptr[r + 1]; k++) {
                int32_t c = col_idx[k];
                if (mask[r] || mask[c]) K[k] = (r == c) ? 1.0 : 0.0;
            }
    }
    return 0;
}

/* Element energies s_e = u_e^T K_e^0 u_e (u_e = u at the element's dofs). */
int oracle_element_energy(int elem, int64_t n_nodes, const double *coords, int64_t n_cells,
                          const int32_t *cells, double nu, int plane_strain, const double *u,
                          double *s) {
    int dim = elem_dim(elem), nen = elem_nen(elem), ldof, i, j;
    int64_t e;
    double xe[3 * MAXNEN], Ke[MAXLDOF * MAXLDOF], ue[MAXLDOF];
    if (dim < 0) return -1;
    (void)n_nodes;
    ldof = dim * nen;
    for (e = 0; e < n_cells; e++) {
        const int32_t *cell = cells + e * nen;
        double acc = 0.0;
        gather_coords(dim, nen, coords, cell, xe);
        oracle_element_ke0(elem, xe, nu, plane_strain, Ke);
        for (i = 0; i < ldof; i++) ue[i] = u[(int64_t)dim * cell[i / dim] + i % dim];
        for (i = 0; i < ldof; i++) {
            double row = 0.0;
            for (j = 0; j < ldof; j++) row += Ke[ldof * i + j] * ue[j];
            acc += ue[i] * row;
        }
        s[e] = acc;
    }
    return 0;
}

/* dc_e = -p rho_e^(p-1) (E0-Emin) u_e^T K_e^0 u_e   (Appendix D). */
int oracle_sensitivity(int elem, int64_t n_nodes, const double *coords, int64_t n_cells,
                       const int32_t *cells, const double *rho, double E0, double Emin, double p,
                       double nu, int plane_strain, const double *u, double *dc) {
    int64_t e;
    int rc = oracle_element_energy(elem, n_nodes, coords, n_cells, cells, nu, plane_strain, u, dc);
    if (rc) return rc;
    for (e = 0; e < n_cells; e++) dc[e] = -simp_dE(rho[e], E0, Emin, p) * dc[e];
    return 0;
}

/* c[0] = sum_e E(rho_e) u_e^T K_e^0 u_e (= u^T K u), ascending e;
 * c[1] = f^T u if f != NULL (Eq. cmpd). */
int oracle_compliance(int elem, int64_t n_nodes, const double *coords, int64_t n_cells,
                      const int32_t *cells, const double *rho, double E0, double Emin, double p,
                      double nu, int plane_strain, const double *u, const double *f, double *c) {
    int dim = elem_dim(elem);
    int64_t e, r;
    double acc = 0.0, *s;
    if (dim < 0) return -1;
    s = (double *)malloc(sizeof(double) * (size_t)(n_cells > 0 ? n_cells : 1));
    if (!s) return -3;
    oracle_element_energy(elem, n_nodes, coords, n_cells, cells, nu, plane_strain, u, s);
    for (e = 0; e < n_cells; e++) acc += simp_E(rho[e], E0, Emin, p) * s[e];
    free(s);
    c[0] = acc;
    if (f) {
        double fu = 0.0;
        for (r = 0; r < dim * n_nodes; r++) fu += f[r] * u[r];
        c[1] = fu;
    }
    return 0;
}

/* Reverse of the assembly map: drho_e = E'(rho_e) sum_ij Kbar[slot(e,i,j)] K_e^0[i][j]. */
int oracle_assemble_backward(int elem, int64_t n_nodes, const double *coords, int64_t n_cells,
                             const int32_t *cells, const double *rho, double E0, double Emin,
                             double p, double nu, int plane_strain, const int64_t *row_ptr,
                             const int32_t *col_idx, const double *Kbar, double *drho) {
    int dim = elem_dim(elem), nen = elem_nen(elem), ldof, i, j;
    int64_t e;
    double xe[3 * MAXNEN], Ke[MAXLDOF * MAXLDOF];
    if (dim < 0) return -1;
    (void)n_nodes;
    ldof = dim * nen;
    for (e = 0; e < n_cells; e++) {
        const int32_t *cell = cells + e * nen;
        double acc = 0.0;
        gather_coords(dim, nen, coords, cell, xe);
        oracle_element_ke0(elem, xe, nu, plane_strain, Ke);
        for (i = 0; i < ldof; i++) {
            int64_t gr = (int64_t)dim * cell[i / dim] + i % dim;
            for (j = 0; j < ldof; j++) {
                int32_t gc = (int32_t)(dim * cell[j / dim] + j % dim);
                int64_t s = find_slot(row_ptr, col_idx, gr, gc);
                if (s < 0) return -2;
                acc += Kbar[s] * Ke[ldof * i + j];
            }
        }
        drho[e] = simp_dE(rho[e], E0, Emin, p) * acc;
    }
    return 0;
}

/* K u for a CSR matrix. */
int oracle_spmv(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *K,
                const double *x, double *y) {
    int64_t r, k;
    for (r = 0; r < n; r++) {
        double s = 0.0;
        for (k = row_ptr[r]; k < row_ptr[r + 1]; k++) s += K[k] * x[col_idx[k]];
        y[r] = s;
    }
    return 0;
}

/* Solve K u = f for a symmetric positive definite CSR matrix by banded
 * Cholesky (K = L L^T with L lower triangular, half-bandwidth bw).
 * band: workspace of n*(bw+1) doubles; band[r*(bw+1) + (c-r+bw)] = L[r][c]. */
int oracle_solve_banded(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *K,
                        const double *f, int64_t bw, double *band, double *u) {
    int64_t r, c, k, w = bw + 1;
#define LB(r_, c_) band[(r_) * w + ((c_) - (r_) + bw)]
    memset(band, 0, sizeof(double) * (size_t)(n * w));
    for (r = 0; r < n; r++)
        for (k = row_ptr[r]; k < row_ptr[r + 1]; k++) {
            c = col_idx[k];
            if (c <= r) {
                if (r - c > bw) return -1;
                LB(r, c) = K[k];
            }
        }
    for (r = 0; r < n; r++) {
        int64_t c0 = r - bw > 0 ? r - bw : 0;
        for (c = c0; c <= r; c++) {
            double s = LB(r, c);
            int64_t k0 = (r - bw > c - bw ? r - bw : c - bw), kk;
            if (k0 < 0) k0 = 0;
            for (kk = k0; kk < c; kk++) s -= LB(r, kk) * LB(c, kk);
            if (c == r) {
                if (s <= 0.0) return -4;
                LB(r, r) = sqrt(s);
            } else {
                LB(r, c) = s / LB(c, c);
            }
        }
    }
    /* forward: L y = f */
    for (r = 0; r < n; r++) {
        double s = f[r];
        int64_t c0 = r - bw > 0 ? r - bw : 0;
        for (c = c0; c < r; c++) s -= LB(r, c) * u[c];
        u[r] = s / LB(r, r);
    }
    /* backward: L^T u = y */
    for (r = n - 1; r >= 0; r--) {
        double s = u[r];
        int64_t c1 = r + bw < n - 1 ? r + bw : n - 1;
        for (c = r + 1; c <= c1; c++) s -= LB(c, r) * u[c];
        u[r] = s / LB(r, r);
    }
#undef LB
    return 0;
}

/* ------------------------------------------------------------------------
 * Multi-threaded variants (OpenMP), used only as the second row of the
 * benchmark's CPU baseline.  They do the arithmetic of oracle_assemble,
 * oracle_element_energy, oracle_sensitivity and oracle_compliance in the
 * same per-value order, so each result is bitwise the serial one:
 *  - assembly: thread t owns a contiguous block of rows holding about 1/T of
 *    the stored entries and walks every element in ascending id, adding only
 *    into its own rows, so every stored value still sums its elements in
 *    ascending id (an element whose nodes fall in two blocks has K_e^0
 *    computed by both threads);
 *  - energies: elements split over threads (s_e is one element's own sum);
 *  - compliance: energies in parallel, then the serial ascending sum.
 * ---------------------------------------------------------------------- */
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* smallest row r in [0, n] with row_ptr[r] >= s */
static int64_t first_row_at(const int64_t *row_ptr, int64_t n, int64_t s) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (row_ptr[mid] >= s) hi = mid; else lo = mid + 1;
    }
    return lo;
}

int oracle_assemble_mt(int elem, int64_t n_nodes, const double *coords, int64_t n_cells,
                       const int32_t *cells, const double *rho, double E0, double Emin, double p,
                       double nu, int plane_strain, const uint8_t *mask, const int64_t *row_ptr,
                       const int32_t *col_idx, double *K) {
    int dim = elem_dim(elem), nen = elem_nen(elem), bad = 0;
    int64_t ndof, nnz;
    if (dim < 0) return -1;
    ndof = dim * n_nodes;
    nnz = row_ptr[ndof];
#pragma omp parallel reduction(| : bad)
    {
        int nt = 1, t = 0, ldof = dim * nen, i, j, a;
        int64_t e, r, k, r0, r1;
        double xe[3 * MAXNEN], Ke[MAXLDOF * MAXLDOF];
#ifdef _OPENMP
        nt = omp_get_num_threads();
        t = omp_get_thread_num();
#endif
        r0 = first_row_at(row_ptr, ndof, nnz * t / nt);
        r1 = t == nt - 1 ? ndof : first_row_at(row_ptr, ndof, nnz * (t + 1) / nt);
        if (r1 > r0) memset(K + row_ptr[r0], 0, sizeof(double) * (size_t)(row_ptr[r1] - row_ptr[r0]));
        for (e = 0; e < n_cells && !bad; e++) {
            const int32_t *cell = cells + e * nen;
            int touch = 0;
            double Ee;
            for (i = 0; i < nen; i++)
                for (a = 0; a < dim; a++) {
                    int64_t gr = (int64_t)dim * cell[i] + a;
                    if (gr >= r0 && gr < r1) touch = 1;
                }
            if (!touch) continue;
            Ee = simp_E(rho[e], E0, Emin, p);
            gather_coords(dim, nen, coords, cell, xe);
            oracle_element_ke0(elem, xe, nu, plane_strain, Ke);
            for (i = 0; i < ldof; i++) {
                int64_t gr = (int64_t)dim * cell[i / dim] + i % dim;
                if (gr < r0 || gr >= r1) continue;
                for (j = 0; j < ldof; j++) {
                    int32_t gc = (int32_t)(dim * cell[j / dim] + j % dim);
                    int64_t s = find_slot(row_ptr, col_idx, gr, gc);
                    if (s < 0) { bad = 1; break; }
                    K[s] += Ee * Ke[ldof * i + j];
                }
            }
        }
        if (mask && !bad) {
            for (r = r0; r < r1; r++)
                for (k = row_ptr[r]; k < row_ptr[r + 1]; k++) {
                    int32_t c = col_idx[k];
                    if (mask[r] || mask[c]) K[k] = (r == c) ? 1.0 : 0.0;
                }
        }
    }
    return bad ? -2 : 0;
}

int oracle_element_energy_mt(int elem, int64_t n_nodes, const double *coords, int64_t n_cells,
                             const int32_t *cells, double nu, int plane_strain, const double *u,
                             double *s) {
    int dim = elem_dim(elem), nen = elem_nen(elem);
    int64_t e;
    if (dim < 0) return -1;
    (void)n_nodes;
#pragma omp parallel for schedule(static)
    for (e = 0; e < n_cells; e++) {
        int ldof = dim * nen, i, j;
        const int32_t *cell = cells + e * nen;
        double xe[3 * MAXNEN], Ke[MAXLDOF * MAXLDOF], ue[MAXLDOF], acc = 0.0;
        gather_coords(dim, nen, coords, cell, xe);
        oracle_element_ke0(elem, xe, nu, plane_strain, Ke);
        for (i = 0; i < ldof; i++) ue[i] = u[(int64_t)dim * cell[i / dim] + i % dim];
        for (i = 0; i < ldof; i++) {
            double row = 0.0;
            for (j = 0; j < ldof; j++) row += Ke[ldof * i + j] * ue[j];
            acc += ue[i] * row;
        }
        s[e] = acc;
    }
    return 0;
}

int oracle_sensitivity_mt(int elem, int64_t n_nodes, const double *coords, int64_t n_cells,
                          const int32_t *cells, const double *rho, double E0, double Emin, double p,
                          double nu, int plane_strain, const double *u, double *dc) {
    int64_t e;
    int rc = oracle_element_energy_mt(elem, n_nodes, coords, n_cells, cells, nu, plane_strain, u, dc);
    if (rc) return rc;
#pragma omp parallel for schedule(static)
    for (e = 0; e < n_cells; e++) dc[e] = -simp_dE(rho[e], E0, Emin, p) * dc[e];
    return 0;
}

int oracle_compliance_mt(int elem, int64_t n_nodes, const double *coords, int64_t n_cells,
                         const int32_t *cells, const double *rho, double E0, double Emin, double p,
                         double nu, int plane_strain, const double *u, const double *f, double *c) {
    int dim = elem_dim(elem);
    int64_t e, r;
    double acc = 0.0, *s;
    if (dim < 0) return -1;
    s = (double *)malloc(sizeof(double) * (size_t)(n_cells > 0 ? n_cells : 1));
    if (!s) return -3;
    oracle_element_energy_mt(elem, n_nodes, coords, n_cells, cells, nu, plane_strain, u, s);
    for (e = 0; e < n_cells; e++) acc += simp_E(rho[e], E0, Emin, p) * s[e];
    free(s);
    c[0] = acc;
    if (f) {
        double fu = 0.0;
        for (r = 0; r < dim * n_nodes; r++) fu += f[r] * u[r];
        c[1] = fu;
    }
    return 0;
}
