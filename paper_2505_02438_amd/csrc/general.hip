// gfx950 kernels of the SIMP stiffness assembly with per-quadrature-point
// geometry (arXiv 2505.02438, Sec. 2.1-2.2; Q1 elements whose map is not
// affine, where the separated form of the fast assembly does not hold).
//
// k_ke_general: the blocks of every element's matrix,
//     Ke[i][j] = E(rho_e) sum_q w_q |det J_q| L(g_i g_j^T) = L(P_ij),
//     P_ij = sum_q c_q g_i g_j^T,  c_q = w_q |det J_q| E(rho_e),
//     g_k = J_q^-T grad phi_k(xi_q),  L(A) = lambda A + mu A^T + mu tr(A) I
// (L is linear, so the per-point sum is taken on P), with one thread per
// node pair i <= j of an element (36 per hexahedron, 10 per quadrilateral);
// block (j, i) is the transpose of block (i, j), so Ke is exactly symmetric.
// The first NQ threads of an element form J_q^-1 and c_q in LDS, and the
// elements of a block are written out as one contiguous range.
// k_energy_general: element energies, sensitivities and the compliance
// partials with the same per-point geometry.
// k_gather_general: one thread per DIM x DIM block of K adds its element
// contributions in ascending element order (the order of a sequential loop
// over elements) and writes the block once.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "kernels.h"

namespace soptx {

namespace {

__device__ __noinline__ double general_pow(double x, double p) { return pow(x, p); }

// E(rho) = Emin + rho^p (E0 - Emin); an integer p by repeated products
__device__ __forceinline__ double simp_modulus(double r, const GenParams &G) {
    double t;
    if (G.ip >= 0) {
        t = 1.0;
        for (int k = 0; k < G.ip; k++) t *= r;
    } else {
        t = general_pow(r, G.p);
    }
    return G.Emin + t * (G.E0 - G.Emin);
}

template <int DIM, int NEN, int NQ>
__global__ __launch_bounds__(256) void k_ke_general(GenParams G) {
    constexpr int NP = NEN * NEN;            // blocks per element
    constexpr int NU = NEN * (NEN + 1) / 2;  // threads per element: pairs i <= j
    constexpr int EPB = 256 / NU;            // elements per block
    constexpr int D2 = DIM * DIM;
    static_assert(NQ <= NU, "the Jacobians take one thread per point");
    __shared__ double sg[EPB][NQ][D2 + 1];  // J_q^-1 (row m: d xi_m / d x), then w_q |det J_q| E
    __shared__ double sq[NQ * NEN * DIM];   // reference gradients at the quadrature points
    __shared__ double so[EPB * NP * D2];    // the block's element matrices, written out contiguously
    for (int x = threadIdx.x; x < NQ * NEN * DIM; x += 256) sq[x] = G.qgrad[x];
    const int le = threadIdx.x / NU, pr = threadIdx.x % NU;
    const int64_t e = (int64_t)blockIdx.x * EPB + le;
    const bool live = le < EPB && e < G.n_cells;
    __syncthreads();
    if (live && pr < NQ) {
        const int q = pr;
        double J[DIM][DIM];
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int m = 0; m < DIM; m++) J[a][m] = 0.0;
        for (int k = 0; k < NEN; k++) {
            const int64_t nd = G.cells[e * NEN + k];
#pragma unroll
            for (int a = 0; a < DIM; a++) {
                const double x = G.coords[nd * DIM + a];
#pragma unroll
                for (int m = 0; m < DIM; m++) J[a][m] += x * sq[(q * NEN + k) * DIM + m];
            }
        }
        double inv[DIM][DIM], det;
        if (DIM == 2) {
            det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            const double id = 1.0 / det;
            inv[0][0] = J[1][1] * id;
            inv[0][1] = -J[0][1] * id;
            inv[1][0] = -J[1][0] * id;
            inv[1][1] = J[0][0] * id;
        } else {
            const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
            const double c01 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
            const double c02 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
            const double c10 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
            const double c11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
            const double c12 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
            const double c20 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
            const double c21 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
            const double c22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            det = J[0][0] * c00 + J[0][1] * c10 + J[0][2] * c20;
            const double id = 1.0 / det;
            inv[0][0] = c00 * id; inv[0][1] = c01 * id; inv[0][2] = c02 * id;
            inv[1][0] = c10 * id; inv[1][1] = c11 * id; inv[1][2] = c12 * id;
            inv[2][0] = c20 * id; inv[2][1] = c21 * id; inv[2][2] = c22 * id;
        }
#pragma unroll
        for (int m = 0; m < DIM; m++)
#pragma unroll
            for (int a = 0; a < DIM; a++) sg[le][q][m * DIM + a] = inv[m][a];
        sg[le][q][D2] = G.qw[q] * fabs(det) * simp_modulus(G.rho[e], G);
    }
    __syncthreads();
    // pair index -> (i, j), i <= j, rows of the upper triangle in order
    int i = 0, r = pr;
    while (r >= NEN - i) { r -= NEN - i; i++; }
    const int j = i + r;
    double P[DIM][DIM];
#pragma unroll
    for (int a = 0; a < DIM; a++)
#pragma unroll
        for (int c = 0; c < DIM; c++) P[a][c] = 0.0;
    if (live) {
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            double gi[DIM], gj[DIM];
#pragma unroll
            for (int a = 0; a < DIM; a++) {
                double si = 0.0, sj = 0.0;
#pragma unroll
                for (int m = 0; m < DIM; m++) {
                    const double gm = sg[le][q][m * DIM + a];
                    si += sq[(q * NEN + i) * DIM + m] * gm;
                    sj += sq[(q * NEN + j) * DIM + m] * gm;
                }
                gi[a] = sg[le][q][D2] * si;
                gj[a] = sj;
            }
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int c = 0; c < DIM; c++) P[a][c] += gi[a] * gj[c];
        }
        double tr = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; a++) tr += P[a][a];
        double *o = so + le * NP * D2;
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int c = 0; c < DIM; c++) {
                const double b = G.lam * P[a][c] + G.mu * P[c][a] + (a == c ? G.mu * tr : 0.0);
                o[(i * NEN + j) * D2 + a * DIM + c] = b;
                if (i != j) o[(j * NEN + i) * D2 + c * DIM + a] = b;
            }
    }
    __syncthreads();
    // the block's elements are consecutive: one contiguous range of ke
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    const int64_t ne = G.n_cells - e0 < EPB ? G.n_cells - e0 : EPB;
    double *dst = G.ke + e0 * NP * D2;
    for (int64_t x = threadIdx.x; x < ne * NP * D2; x += 256) __builtin_nontemporal_store(so[x], dst + x);
}

template <int DIM>
__global__ __launch_bounds__(256) void k_gather_general(GenParams G) {
    constexpr int D2 = DIM * DIM;
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= G.n_blocks) return;
    const int64_t I = G.gnode[b];
    const int32_t base = G.row_ptr[DIM * I];
    const int32_t rl = G.row_ptr[DIM * I + 1] - base;
    const int64_t q = b - base / D2;
    double acc[D2];
#pragma unroll
    for (int t = 0; t < D2; t++) acc[t] = 0.0;
    for (int32_t k = G.gptr[b]; k < G.gptr[b + 1]; k++) {
        const double *s = G.ke + (int64_t)G.gent[k] * D2;
#pragma unroll
        for (int t = 0; t < D2; t++) acc[t] += s[t];
    }
#pragma unroll
    for (int a = 0; a < DIM; a++)
#pragma unroll
        for (int c = 0; c < DIM; c++) G.K[base + (int64_t)a * rl + DIM * q + c] = acc[a * DIM + c];
}

// Element energies with the Jacobian at every Gauss point, one thread per
// element: s_e = sum_q w_q |det J_q| (lambda tr(eps)^2 + 2 mu eps:eps), eps
// the symmetric part of grad u = sum_k u_k g_k^T (equal to u_e^T K_e^0 u_e
// for the same rule), dc_e = -p rho^(p-1) (E0 - Emin) s_e, and block
// partials of c = sum_e E(rho_e) s_e and of f^T u in a fixed order.
template <int DIM, int NEN, int NQ>
__global__ __launch_bounds__(256) void k_energy_general(GenEnergyParams P) {
    __shared__ double red[256];
    __shared__ double sq[NQ * NEN * DIM];
    for (int x = threadIdx.x; x < NQ * NEN * DIM; x += 256) sq[x] = P.qgrad[x];
    __syncthreads();
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double cpart = 0.0;
    if (e < P.n_cells) {
        double x[NEN][DIM], ue[NEN][DIM];
        for (int k = 0; k < NEN; k++) {
            const int64_t nd = P.cells[e * NEN + k];
#pragma unroll
            for (int a = 0; a < DIM; a++) {
                x[k][a] = P.coords[nd * DIM + a];
                ue[k][a] = P.u[nd * DIM + a];
            }
        }
        double s = 0.0;
        for (int q = 0; q < NQ; q++) {
            double J[DIM][DIM], Hr[DIM][DIM];  // dx_a / dxi_m and du_a / dxi_m
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int m = 0; m < DIM; m++) J[a][m] = Hr[a][m] = 0.0;
            for (int k = 0; k < NEN; k++)
#pragma unroll
                for (int m = 0; m < DIM; m++) {
                    const double gm = sq[(q * NEN + k) * DIM + m];
#pragma unroll
                    for (int a = 0; a < DIM; a++) {
                        J[a][m] += x[k][a] * gm;
                        Hr[a][m] += ue[k][a] * gm;
                    }
                }
            double inv[DIM][DIM], det;
            if (DIM == 2) {
                det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
                const double id = 1.0 / det;
                inv[0][0] = J[1][1] * id;
                inv[0][1] = -J[0][1] * id;
                inv[1][0] = -J[1][0] * id;
                inv[1][1] = J[0][0] * id;
            } else {
                const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
                const double c01 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
                const double c02 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
                const double c10 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
                const double c11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
                const double c12 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
                const double c20 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
                const double c21 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
                const double c22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
                det = J[0][0] * c00 + J[0][1] * c10 + J[0][2] * c20;
                const double id = 1.0 / det;
                inv[0][0] = c00 * id; inv[0][1] = c01 * id; inv[0][2] = c02 * id;
                inv[1][0] = c10 * id; inv[1][1] = c11 * id; inv[1][2] = c12 * id;
                inv[2][0] = c20 * id; inv[2][1] = c21 * id; inv[2][2] = c22 * id;
            }
            // grad u = Hr J^-1, then the energy density of its symmetric part
            double H[DIM][DIM];
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int b = 0; b < DIM; b++) {
                    double t = 0.0;
#pragma unroll
                    for (int m = 0; m < DIM; m++) t += Hr[a][m] * inv[m][b];
                    H[a][b] = t;
                }
            double tr = 0.0, ee = 0.0;
#pragma unroll
            for (int a = 0; a < DIM; a++) {
                tr += H[a][a];
#pragma unroll
                for (int b = 0; b < DIM; b++) {
                    const double eab = 0.5 * (H[a][b] + H[b][a]);
                    ee += eab * eab;
                }
            }
            s += P.qw[q] * fabs(det) * (P.lam * tr * tr + 2.0 * P.mu * ee);
        }
        const double r = P.rho[e];
        double rp1 = 1.0;  // rho^(p - 1)
        if (P.ip >= 1) {
            for (int k = 0; k < P.ip - 1; k++) rp1 *= r;
        } else {
            rp1 = general_pow(r, P.p - 1.0);
        }
        const double E = P.Emin + rp1 * r * (P.E0 - P.Emin);
        if (P.dc) P.dc[e] = -P.p * rp1 * (P.E0 - P.Emin) * s;
        cpart = E * s;
    }
    if (!P.partials) return;
    double fpart = 0.0;
    if (P.f)
        for (int64_t rr = (int64_t)blockIdx.x * 256 + threadIdx.x; rr < P.ndof; rr += (int64_t)gridDim.x * 256)
            fpart += P.f[rr] * P.u[rr];
    // fixed-order block sums (every thread reaches them)
    red[threadIdx.x] = cpart;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    const double bc = red[0];
    __syncthreads();
    red[threadIdx.x] = fpart;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        P.partials[blockIdx.x] = bc;
        P.partials[gridDim.x + blockIdx.x] = P.f ? red[0] : 0.0;
    }
}

// Elements with more node pairs than a block has threads (Q2 hexahedra: 729
// pairs, 27 Gauss points): one element per block.  The block stages the
// node coordinates, then J at the points (a thread per entry), J_q^-1 and
// c_q = w_q |det J_q| E (a thread per point), then every physical gradient
// g_k(xi_q) (a thread per (q, k)), all in LDS.  A thread per two neighbouring
// node pairs (i, j), (i, j + 1), i <= j, of the upper triangle (196 threads
// for a Q2 hexahedron; g_i is read once for both) accumulates
// P = sum_q c_q g_i g_j^T and forms the block
//     lambda P + mu P^T + mu tr(P) I
// (the same sum as k_ke_general's per-point form, regrouped) into an LDS
// stage of the upper triangle's blocks (27.2 KB for a Q2 hexahedron, so that
// three workgroups fit a CU).  The element's full matrix is written out as
// one contiguous range, block (j, i) read as the transpose of block (i, j):
// the element matrix is exactly symmetric.
template <int NEN, int NQ>
__global__ __launch_bounds__(256) void k_ke_general_wide(GenParams G) {
    constexpr int DIM = 3, D2 = 9, NP = NEN * NEN, NU = NEN * (NEN + 1) / 2;
    static_assert(NQ * D2 <= 256 && NQ <= 256, "one thread per Jacobian entry");
    __shared__ double sx[NEN * DIM];       // node coordinates
    __shared__ double sJ[NQ * D2];         // J_q, entry (a, m) = d x_a / d xi_m
    __shared__ double sg[NQ][D2 + 1];      // J_q^-1 (row m: d xi_m / d x), then c_q
    __shared__ double sp[NQ * NEN * DIM];  // physical gradients at the points, [q][k][a]
    __shared__ double so[NU * D2];         // the element matrix's blocks i <= j
    const int64_t e = blockIdx.x;
    const int t = threadIdx.x;
    for (int x = t; x < NEN * DIM; x += 256) sx[x] = G.coords[(int64_t)G.cells[e * NEN + x / DIM] * DIM + x % DIM];
    __syncthreads();
    if (t < NQ * D2) {
        const int q = t / D2, a = (t % D2) / DIM, m = t % DIM;
        double s = 0.0;
        for (int k = 0; k < NEN; k++) s += sx[k * DIM + a] * G.qgrad[(q * NEN + k) * DIM + m];
        sJ[t] = s;
    }
    __syncthreads();
    if (t < NQ) {
        const int q = t;
        const double *J = sJ + q * D2;  // J[a * 3 + m]
        const double c00 = J[4] * J[8] - J[5] * J[7];
        const double c01 = J[2] * J[7] - J[1] * J[8];
        const double c02 = J[1] * J[5] - J[2] * J[4];
        const double c10 = J[5] * J[6] - J[3] * J[8];
        const double c11 = J[0] * J[8] - J[2] * J[6];
        const double c12 = J[2] * J[3] - J[0] * J[5];
        const double c20 = J[3] * J[7] - J[4] * J[6];
        const double c21 = J[1] * J[6] - J[0] * J[7];
        const double c22 = J[0] * J[4] - J[1] * J[3];
        const double det = J[0] * c00 + J[1] * c10 + J[2] * c20;
        const double id = 1.0 / det;
        sg[q][0] = c00 * id; sg[q][1] = c01 * id; sg[q][2] = c02 * id;
        sg[q][3] = c10 * id; sg[q][4] = c11 * id; sg[q][5] = c12 * id;
        sg[q][6] = c20 * id; sg[q][7] = c21 * id; sg[q][8] = c22 * id;
        sg[q][D2] = G.qw[q] * fabs(det) * simp_modulus(G.rho[e], G);
    }
    __syncthreads();
    for (int x = t; x < NQ * NEN; x += 256) {
        const int q = x / NEN, k = x % NEN;
#pragma unroll
        for (int a = 0; a < DIM; a++) {
            double g = 0.0;
#pragma unroll
            for (int m = 0; m < DIM; m++) g += G.qgrad[(q * NEN + k) * DIM + m] * sg[q][m * DIM + a];
            sp[x * DIM + a] = g;
        }
    }
    __syncthreads();
    int ns = 0;  // strips of two neighbouring pairs (i, j), (i, j + 1) in the upper triangle
    for (int r = 0; r < NEN; r++) ns += (NEN - r + 1) / 2;
    for (int pu = t; pu < ns; pu += 256) {
        int i = 0, r = pu;
        while (r >= (NEN - i + 1) / 2) { r -= (NEN - i + 1) / 2; i++; }
        const int j0 = i + 2 * r;
        const bool two = j0 + 1 < NEN;
        const int j1 = two ? j0 + 1 : j0;
        double P0[DIM][DIM], P1[DIM][DIM];
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int c = 0; c < DIM; c++) P0[a][c] = P1[a][c] = 0.0;
#pragma unroll 3
        for (int q = 0; q < NQ; q++) {
            const double cq = sg[q][D2];
            double wi[DIM], g0[DIM], g1[DIM];
#pragma unroll
            for (int a = 0; a < DIM; a++) {
                wi[a] = cq * sp[(q * NEN + i) * DIM + a];
                g0[a] = sp[(q * NEN + j0) * DIM + a];
                g1[a] = sp[(q * NEN + j1) * DIM + a];
            }
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int c = 0; c < DIM; c++) {
                    P0[a][c] += wi[a] * g0[c];
                    P1[a][c] += wi[a] * g1[c];
                }
        }
#pragma unroll
        for (int h = 0; h < 2; h++) {
            if (h == 1 && !two) break;
            const int j = h ? j1 : j0;
            double (*P)[DIM] = h ? P1 : P0;
            const double mtr = G.mu * (P[0][0] + P[1][1] + P[2][2]);
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int c = 0; c < DIM; c++) {
                    const double b = G.lam * P[a][c] + G.mu * P[c][a] + (a == c ? mtr : 0.0);
                    so[(i * NEN - i * (i - 1) / 2 + (j - i)) * D2 + a * DIM + c] = b;
                }
        }
    }
    __syncthreads();
    double *dst = G.ke + e * NP * D2;
    for (int x = t; x < NP * D2; x += 256) {
        const int blk = x / D2, u = x % D2, i = blk / NEN, j = blk % NEN, a = u / DIM, c = u % DIM;
        const double v = i <= j ? so[(i * NEN - i * (i - 1) / 2 + (j - i)) * D2 + a * DIM + c]
                                : so[(j * NEN - j * (j - 1) / 2 + (i - j)) * D2 + c * DIM + a];
        __builtin_nontemporal_store(v, dst + x);
    }
}

// Element energies of Q2 hexahedra: kEnergyWideElems elements per block, each
// of the 4 waves takes kEnergyWideElems / 4 of them in turn.  Per element the
// node coordinates and displacements go to LDS, lane q < NQ forms the
// point's term w_q |det J_q| (lambda tr(eps)^2 + 2 mu eps:eps) with the same
// arithmetic as k_energy_general, and lane 0 adds the terms in ascending q.
// Block partials: the block's element terms E s_e in ascending element
// order, and f^T u as in k_energy_general.
template <int NEN, int NQ>
__global__ __launch_bounds__(256) void k_energy_general_wide(GenEnergyParams P) {
    constexpr int DIM = 3, EPB = kEnergyWideElems, PER_WAVE = EPB / 4;
    __shared__ double red[256];
    __shared__ double cp[EPB];
    __shared__ double nx[4][NEN][2 * DIM];  // per wave: x then u of each node
    __shared__ double sv[4][NQ];
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int it = 0; it < PER_WAVE; it++) {
        const int el = w * PER_WAVE + it;
        const int64_t e = (int64_t)blockIdx.x * EPB + el;
        const bool live = e < P.n_cells;
        if (live && lane < NEN) {
            const int64_t nd = P.cells[e * NEN + lane];
#pragma unroll
            for (int a = 0; a < DIM; a++) {
                nx[w][lane][a] = P.coords[nd * DIM + a];
                nx[w][lane][DIM + a] = P.u[nd * DIM + a];
            }
        }
        __syncthreads();
        if (live && lane < NQ) {
            const int q = lane;
            double J[DIM][DIM], Hr[DIM][DIM];
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int m = 0; m < DIM; m++) J[a][m] = Hr[a][m] = 0.0;
            for (int k = 0; k < NEN; k++)
#pragma unroll
                for (int m = 0; m < DIM; m++) {
                    const double gm = P.qgrad[(q * NEN + k) * DIM + m];
#pragma unroll
                    for (int a = 0; a < DIM; a++) {
                        J[a][m] += nx[w][k][a] * gm;
                        Hr[a][m] += nx[w][k][DIM + a] * gm;
                    }
                }
            const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
            const double c01 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
            const double c02 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
            const double c10 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
            const double c11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
            const double c12 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
            const double c20 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
            const double c21 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
            const double c22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            const double det = J[0][0] * c00 + J[0][1] * c10 + J[0][2] * c20;
            const double id = 1.0 / det;
            const double inv[DIM][DIM] = {{c00 * id, c01 * id, c02 * id},
                                          {c10 * id, c11 * id, c12 * id},
                                          {c20 * id, c21 * id, c22 * id}};
            double H[DIM][DIM];
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int b = 0; b < DIM; b++) {
                    double t = 0.0;
#pragma unroll
                    for (int m = 0; m < DIM; m++) t += Hr[a][m] * inv[m][b];
                    H[a][b] = t;
                }
            double tr = 0.0, ee = 0.0;
#pragma unroll
            for (int a = 0; a < DIM; a++) {
                tr += H[a][a];
#pragma unroll
                for (int b = 0; b < DIM; b++) {
                    const double eab = 0.5 * (H[a][b] + H[b][a]);
                    ee += eab * eab;
                }
            }
            sv[w][q] = P.qw[q] * fabs(det) * (P.lam * tr * tr + 2.0 * P.mu * ee);
        }
        __syncthreads();
        if (lane == 0) {
            double cpart = 0.0;
            if (live) {
                double s = 0.0;
                for (int q = 0; q < NQ; q++) s += sv[w][q];
                const double r = P.rho[e];
                double rp1 = 1.0;  // rho^(p - 1)
                if (P.ip >= 1) {
                    for (int k = 0; k < P.ip - 1; k++) rp1 *= r;
                } else {
                    rp1 = general_pow(r, P.p - 1.0);
                }
                const double E = P.Emin + rp1 * r * (P.E0 - P.Emin);
                if (P.dc) P.dc[e] = -P.p * rp1 * (P.E0 - P.Emin) * s;
                cpart = E * s;
            }
            cp[el] = cpart;
        }
        // the next element's LDS writes come after the next barrier, which
        // lane 0 reaches only once it has read sv
    }
    if (!P.partials) return;
    double fpart = 0.0;
    if (P.f)
        for (int64_t rr = (int64_t)blockIdx.x * 256 + threadIdx.x; rr < P.ndof; rr += (int64_t)gridDim.x * 256)
            fpart += P.f[rr] * P.u[rr];
    red[threadIdx.x] = fpart;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double bc = 0.0;
        for (int k = 0; k < EPB; k++) bc += cp[k];
        P.partials[blockIdx.x] = bc;
        P.partials[gridDim.x + blockIdx.x] = P.f ? red[0] : 0.0;
    }
}

template <int NEN, int NQ>
hipError_t launch_energy_wide(const GenEnergyParams &P, hipStream_t st) {
    if (P.nq != NQ) return hipErrorInvalidValue;
    const unsigned g = (unsigned)((P.n_cells + kEnergyWideElems - 1) / kEnergyWideElems);
    hipLaunchKernelGGL((k_energy_general_wide<NEN, NQ>), dim3(g > 0 ? g : 1), dim3(256), 0, st, P);
    return hipGetLastError();
}

template <int NEN, int NQ>
hipError_t launch_wide(const GenParams &G, hipStream_t st) {
    if (G.nq != NQ) return hipErrorInvalidValue;
    if (G.n_cells > 0) {
        hipLaunchKernelGGL((k_ke_general_wide<NEN, NQ>), dim3((unsigned)G.n_cells), dim3(256), 0, st, G);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (G.n_blocks > 0)
        hipLaunchKernelGGL(k_gather_general<3>, dim3((unsigned)((G.n_blocks + 255) / 256)), dim3(256), 0, st, G);
    return hipGetLastError();
}

template <int DIM, int NEN, int NQ>
hipError_t launch_energy_t(const GenEnergyParams &P, hipStream_t st) {
    if (P.nq != NQ) return hipErrorInvalidValue;
    const unsigned g = (unsigned)((P.n_cells + 255) / 256);
    hipLaunchKernelGGL((k_energy_general<DIM, NEN, NQ>), dim3(g > 0 ? g : 1), dim3(256), 0, st, P);
    return hipGetLastError();
}

template <int DIM, int NEN, int NQ>
hipError_t launch_t(const GenParams &G, hipStream_t st) {
    constexpr int EPB = 256 / (NEN * (NEN + 1) / 2);
    if (G.nq != NQ) return hipErrorInvalidValue;
    if (G.n_cells > 0) {
        hipLaunchKernelGGL((k_ke_general<DIM, NEN, NQ>), dim3((unsigned)((G.n_cells + EPB - 1) / EPB)), dim3(256), 0,
                           st, G);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (G.n_blocks > 0)
        hipLaunchKernelGGL(k_gather_general<DIM>, dim3((unsigned)((G.n_blocks + 255) / 256)), dim3(256), 0, st, G);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_energy_general(int elem, const GenEnergyParams &P, hipStream_t st) {
    if (elem == SOPTX_HEX8) return launch_energy_t<3, 8, 8>(P, st);
    if (elem == SOPTX_HEX27) return launch_energy_wide<27, 27>(P, st);
    if (elem == SOPTX_QUAD4) return launch_energy_t<2, 4, 4>(P, st);
    return hipErrorInvalidValue;
}

hipError_t launch_assemble_general(int elem, const GenParams &G, hipStream_t st) {
    if (elem == SOPTX_HEX8) return launch_t<3, 8, 8>(G, st);
    if (elem == SOPTX_HEX27) return launch_wide<27, 27>(G, st);
    if (elem == SOPTX_QUAD4) return launch_t<2, 4, 4>(G, st);
    return hipErrorInvalidValue;
}

}  // namespace soptx
