// gfx950 kernels for SIMP assembly, element energies, compliance and the
// assembly backward (arXiv 2505.02438: Sec. 2.1 SIMP, Sec. 2.2 Eq. cmpd,
// Sec. 5.5 fast assembly, Appendix D sensitivity).
//
// Element matrix in separated ("fast assembly") form.  For an affine element
// with G = J^-1 (G[m][a] = d xi_m / d x_a) and the reference tensor
// M_ij[m][n] = int_ref d_m phi_i d_n phi_j, the block (i, j) of K_e^0 is
//     K_e^0(i,j) = |det J| L(A_ij),  A_ij = G^T M_ij G,
//     L(A) = lambda A + mu A^T + mu tr(A) I
// (the isotropic form lambda div u div v + 2 mu eps(u):eps(v) written per
// block; plane stress uses lambda* = E nu / (1 - nu^2)).  L is linear, so the
// assembled block is L applied to sum_e E(rho_e) |det J_e| A_ij(e): every
// element contribution costs two 3x3x3 products (T = M_ij G', A += G'^T T with
// G' = sqrt(E |det J|) G) and L is applied once per stored block.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "kernels.h"

namespace soptx {

namespace {

__device__ __forceinline__ double simp_pow(double x, double p, int ip) {
    if (ip >= 0) {
        double r = 1.0;
        for (int k = 0; k < ip; k++) r *= x;
        return r;
    }
    return pow(x, p);
}

template <int PREC>
__device__ __forceinline__ double load_rho(const void *rho, int64_t e) {
    if (PREC == kF64) return static_cast<const double *>(rho)[e];
    return (double)static_cast<const float *>(rho)[e];
}

template <int PREC>
__device__ __forceinline__ void store_out(void *out, int64_t e, double v) {
    if (PREC == kF64) static_cast<double *>(out)[e] = v;
    else static_cast<float *>(out)[e] = (float)v;
}

// round-to-nearest-even to bfloat16, kept in a float
__device__ __forceinline__ float bf16_round(float x) {
    uint32_t u = __float_as_uint(x);
    uint32_t r = ((u >> 16) & 1u) + 0x7fffu;
    return __uint_as_float((u + r) & 0xffff0000u);
}

template <int PREC> struct CT { using T = float; };
template <> struct CT<kF64> { using T = double; };

__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

}  // namespace

// ------------------------------------------------------------------ assembly
//
// One workgroup = one group of up to 64 nodes sharing a connectivity
// signature; lane l of every wave is node grp_nodes[g][l]; wave w stores the
// neighbour positions [sig_wave[w], sig_wave[w+1]) of the row block of its
// node.  Element data of the group (G' per element) is staged once in LDS.
// Summation order of a stored block: the signature's contribution order
// (elements ascending within the block), fixed by the mesh.
template <int DIM, int NEN, int PREC>
__global__ __launch_bounds__(256) void k_assemble(AsmParams P) {
    using T = typename CT<PREC>::T;
    constexpr int D2 = DIM * DIM;
    extern __shared__ __align__(16) unsigned char smem[];
    T *sG = reinterpret_cast<T *>(smem);                          // [D2][emax]
    int32_t *sgid = reinterpret_cast<int32_t *>(sG + D2 * P.emax);  // [emax]
    uint16_t *sn2l = reinterpret_cast<uint16_t *>(sgid + P.emax);    // [kmax][64]

    const int g = blockIdx.x;
    const int sig = P.grp_info[5 * g + 0];
    const int nn = P.grp_info[5 * g + 1];
    const int eoff = P.grp_info[5 * g + 2];
    const int ne = P.grp_info[5 * g + 3];
    const int n2loff = P.grp_info[5 * g + 4];
    const int K = P.sig_info[4 * sig + 0];
    const int posoff = P.sig_info[4 * sig + 2];
    const int woff = P.sig_info[4 * sig + 3];
    const int tid = threadIdx.x;
    const int64_t NC = P.n_cells;

    for (int t = tid; t < ne; t += 256) {
        const int e = P.grp_elems[eoff + t];
        const double r = load_rho<PREC>(P.rho, e);
        const double E = P.Emin + simp_pow(r, P.p, P.ip) * (P.E0 - P.Emin);
        const double q = sqrt(E * P.geo[(int64_t)D2 * NC + e]);
#pragma unroll
        for (int c = 0; c < D2; c++) {
            sG[c * P.emax + t] = (T)(q * P.geo[(int64_t)c * NC + e]);
        }
        sgid[t] = e;
    }
    for (int t = tid; t < K * 64; t += 256) sn2l[t] = P.grp_n2l[n2loff + t];
    __syncthreads();

    const int lane = tid & 63;
    const int w = wave_uniform(tid >> 6);
    if (lane >= nn) return;
    const int I = P.grp_nodes[64 * g + lane];
    const int base = P.row_ptr[DIM * I];
    const int rowlen = P.row_ptr[DIM * I + 1] - base;
    const int p0 = P.sig_wave[woff + w], p1 = P.sig_wave[woff + w + 1];

    for (int p = p0; p < p1; p++) {
        double acc[DIM][DIM];
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int b = 0; b < DIM; b++) acc[a][b] = 0.0;
        const int c0 = P.sig_pos_ptr[posoff + p], c1 = P.sig_pos_ptr[posoff + p + 1];
        for (int t = c0; t < c1; t++) {
            const int pk = P.sig_contrib[t];
            const int k = pk >> 16, i = (pk >> 8) & 255, j = pk & 255;
            const int le = sn2l[k * 64 + lane];
            T G[DIM][DIM];
#pragma unroll
            for (int m = 0; m < DIM; m++)
#pragma unroll
                for (int a = 0; a < DIM; a++) G[m][a] = sG[(m * DIM + a) * P.emax + le];
            const int mij = (i * NEN + j) * D2;
            T Tm[DIM][DIM];
            if (PREC == kF64) {
                const double *Mij = P.M + mij;
#pragma unroll
                for (int m = 0; m < DIM; m++)
#pragma unroll
                    for (int b = 0; b < DIM; b++) {
                        double s = 0.0;
#pragma unroll
                        for (int n = 0; n < DIM; n++) s += Mij[m * DIM + n] * (double)G[n][b];
                        Tm[m][b] = (T)s;
                    }
#pragma unroll
                for (int a = 0; a < DIM; a++)
#pragma unroll
                    for (int b = 0; b < DIM; b++)
#pragma unroll
                        for (int m = 0; m < DIM; m++) acc[a][b] += (double)G[m][a] * (double)Tm[m][b];
            } else if (PREC == kF32) {
                const float *Mij = P.M32 + mij;
#pragma unroll
                for (int m = 0; m < DIM; m++)
#pragma unroll
                    for (int b = 0; b < DIM; b++) {
                        float s = 0.0f;
#pragma unroll
                        for (int n = 0; n < DIM; n++) s += Mij[m * DIM + n] * (float)G[n][b];
                        Tm[m][b] = s;
                    }
#pragma unroll
                for (int a = 0; a < DIM; a++)
#pragma unroll
                    for (int b = 0; b < DIM; b++) {
                        float s = 0.0f;
#pragma unroll
                        for (int m = 0; m < DIM; m++) s += (float)G[m][a] * (float)Tm[m][b];
                        acc[a][b] += (double)s;
                    }
            } else {
                // bf16 inputs, fp32 accumulation: A[a][b] = sum_mn M[m][n] W[m,a][n,b]
                // with both GEMM operands rounded to bf16, W = G'[m][a] G'[n][b]
                const float *Mij = P.Mbf + mij;
#pragma unroll
                for (int a = 0; a < DIM; a++)
#pragma unroll
                    for (int b = 0; b < DIM; b++) {
                        float s = 0.0f;
#pragma unroll
                        for (int m = 0; m < DIM; m++)
#pragma unroll
                            for (int n = 0; n < DIM; n++)
                                s += Mij[m * DIM + n] * bf16_round((float)G[m][a] * (float)G[n][b]);
                        acc[a][b] += (double)s;
                    }
            }
        }
        double tr = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; a++) tr += acc[a][a];
        double out[DIM][DIM];
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int b = 0; b < DIM; b++)
                out[a][b] = P.lam * acc[a][b] + P.mu * acc[b][a] + (a == b ? P.mu * tr : 0.0);
        if (P.mask) {
            // column node of this position: node j of the first contributing element
            const int pk = P.sig_contrib[c0];
            const int k = pk >> 16, j = pk & 255;
            const int e = sgid[sn2l[k * 64 + lane]];
            const int Jn = P.cells[(int64_t)e * NEN + j];
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int b = 0; b < DIM; b++) {
                    const int r = DIM * I + a, c = DIM * Jn + b;
                    if (P.mask[r] | P.mask[c]) out[a][b] = (r == c) ? 1.0 : 0.0;
                }
        }
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int b = 0; b < DIM; b++) P.K[base + a * rowlen + DIM * p + b] = out[a][b];
    }
}

// ------------------------------------------------------- element energies
//
// s_e = u_e^T K_e^0 u_e evaluated as the strain energy sum_q w_q |det J|
// (lambda tr(eps)^2 + 2 mu eps:eps) at the reference quadrature points (exact
// for affine elements; the same quadratic form as u_e^T K_e^0 u_e).
// Writes dc_e = -E'(rho_e) s_e and a fixed-order block partial of
// sum_e E(rho_e) s_e.  In the reduced-precision forms the element's rigid
// motion (translation of node 0 and the rotation of the centroid gradient) is
// removed in FP64 first; it is in the null space of K_e^0, so s_e is unchanged
// in exact arithmetic while the FP32 part sees only the deforming part.
template <int DIM, int NEN, int NQ, int PREC>
__global__ __launch_bounds__(256) void k_energy(EnergyParams P) {
    __shared__ double red[256];
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t NC = P.n_cells;
    constexpr int D2 = DIM * DIM;
    double cpart = 0.0;
    if (e < NC) {
        double G[DIM][DIM];
#pragma unroll
        for (int m = 0; m < DIM; m++)
#pragma unroll
            for (int a = 0; a < DIM; a++) G[m][a] = P.geo[(int64_t)(m * DIM + a) * NC + e];
        const double det = P.geo[(int64_t)D2 * NC + e];
        double u[NEN][DIM];
#pragma unroll
        for (int i = 0; i < NEN; i++) {
            const int n = P.cells[e * NEN + i];
#pragma unroll
            for (int a = 0; a < DIM; a++) u[i][a] = P.u[(int64_t)DIM * n + a];
        }
        double s = 0.0;
        if (PREC == kF64) {
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                const double *dq = P.qgrad + q * NEN * DIM;
                double gr[DIM][DIM];  // reference gradient d u_a / d xi_m
#pragma unroll
                for (int a = 0; a < DIM; a++)
#pragma unroll
                    for (int m = 0; m < DIM; m++) {
                        double t = 0.0;
#pragma unroll
                        for (int i = 0; i < NEN; i++) t += u[i][a] * dq[i * DIM + m];
                        gr[a][m] = t;
                    }
                double eps[DIM][DIM];
#pragma unroll
                for (int a = 0; a < DIM; a++)
#pragma unroll
                    for (int b = 0; b < DIM; b++) {
                        double t = 0.0;
#pragma unroll
                        for (int m = 0; m < DIM; m++) t += gr[a][m] * G[m][b];
                        eps[a][b] = t;
                    }
                double tr = 0.0, ee = 0.0;
#pragma unroll
                for (int a = 0; a < DIM; a++) {
                    tr += eps[a][a];
                    ee += eps[a][a] * eps[a][a];
#pragma unroll
                    for (int b = a + 1; b < DIM; b++) {
                        const double h = 0.5 * (eps[a][b] + eps[b][a]);
                        ee += 2.0 * h * h;
                    }
                }
                s += P.qw[q] * (P.lam * tr * tr + 2.0 * P.mu * ee);
            }
        } else {
            // FP64: remove translation (node 0) and the centroid rotation
            double w[NEN][DIM];
#pragma unroll
            for (int i = 0; i < NEN; i++)
#pragma unroll
                for (int a = 0; a < DIM; a++) w[i][a] = u[i][a] - u[0][a];
            const double *dc = P.cgrad;  // reference gradients at the centroid
            double gx[DIM][DIM];         // physical gradient at the centroid
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int b = 0; b < DIM; b++) {
                    double t = 0.0;
#pragma unroll
                    for (int m = 0; m < DIM; m++) {
                        double r = 0.0;
#pragma unroll
                        for (int i = 0; i < NEN; i++) r += w[i][a] * dc[i * DIM + m];
                        t += r * G[m][b];
                    }
                    gx[a][b] = t;
                }
            // x_i - x_0 = J xi_i, J = G^-1; W J xi_i with W = skew(gx)
            double J[DIM][DIM];
            if (DIM == 2) {
                const double d = G[0][0] * G[1][1] - G[0][1] * G[1][0];
                J[0][0] = G[1][1] / d; J[0][1] = -G[0][1] / d;
                J[1][0] = -G[1][0] / d; J[1][1] = G[0][0] / d;
            } else {
                // J = G^-1, i.e. (det J) * adj(G) with 1/det(G) = det J
#pragma unroll
                for (int a = 0; a < DIM; a++)
#pragma unroll
                    for (int m = 0; m < DIM; m++) {
                        const int a1 = (m + 1) % 3, a2 = (m + 2) % 3, b1 = (a + 1) % 3, b2 = (a + 2) % 3;
                        J[a][m] = det * (G[a1][b1] * G[a2][b2] - G[a1][b2] * G[a2][b1]);
                    }
            }
            double WJ[DIM][DIM];
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int m = 0; m < DIM; m++) {
                    double t = 0.0;
#pragma unroll
                    for (int b = 0; b < DIM; b++) t += 0.5 * (gx[a][b] - gx[b][a]) * J[b][m];
                    WJ[a][m] = t;
                }
            float wf[NEN][DIM];
#pragma unroll
            for (int i = 0; i < NEN; i++)
#pragma unroll
                for (int a = 0; a < DIM; a++) {
                    double t = w[i][a];
#pragma unroll
                    for (int m = 0; m < DIM; m++) t -= WJ[a][m] * P.xref[i * DIM + m];
                    wf[i][a] = (float)t;
                }
            float Gf[DIM][DIM];
#pragma unroll
            for (int m = 0; m < DIM; m++)
#pragma unroll
                for (int a = 0; a < DIM; a++) Gf[m][a] = (float)G[m][a];
            float sf = 0.0f;
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                const float *dq = P.qgrad32 + q * NEN * DIM;
                float gr[DIM][DIM];
#pragma unroll
                for (int a = 0; a < DIM; a++)
#pragma unroll
                    for (int m = 0; m < DIM; m++) {
                        float t = 0.0f;
#pragma unroll
                        for (int i = 0; i < NEN; i++) t += wf[i][a] * dq[i * DIM + m];
                        gr[a][m] = t;
                    }
                float eps[DIM][DIM];
#pragma unroll
                for (int a = 0; a < DIM; a++)
#pragma unroll
                    for (int b = 0; b < DIM; b++) {
                        float t = 0.0f;
#pragma unroll
                        for (int m = 0; m < DIM; m++) t += gr[a][m] * Gf[m][b];
                        eps[a][b] = t;
                    }
                float tr = 0.0f, ee = 0.0f;
#pragma unroll
                for (int a = 0; a < DIM; a++) {
                    tr += eps[a][a];
                    ee += eps[a][a] * eps[a][a];
#pragma unroll
                    for (int b = a + 1; b < DIM; b++) {
                        const float h = 0.5f * (eps[a][b] + eps[b][a]);
                        ee += 2.0f * h * h;
                    }
                }
                sf += (float)P.qw[q] * ((float)P.lam * tr * tr + 2.0f * (float)P.mu * ee);
            }
            s = (double)sf;
        }
        s *= det;
        const double r = load_rho<PREC>(P.rho, e);
        const double rp1 = simp_pow(r, P.p - 1.0, P.ip >= 1 ? P.ip - 1 : -1);
        const double E = P.Emin + rp1 * r * (P.E0 - P.Emin);
        if (P.dc) store_out<PREC>(P.dc, e, -P.p * rp1 * (P.E0 - P.Emin) * s);
        cpart = E * s;
    }
    if (P.partials) {
        red[threadIdx.x] = cpart;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) P.partials[blockIdx.x] = red[0];
    }
}

// f^T u partials: fixed grid, grid-stride, fixed tree per block
__global__ __launch_bounds__(256) void k_dot_partials(const double *__restrict__ f,
                                                      const double *__restrict__ u, int64_t n,
                                                      double *partials) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256)
        s += f[r] * u[r];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// c[0] = sum of p0[0:n0] (0 when n0 == 0); c[1] = sum of p1[0:n1] when p1 is
// given.  Fixed order: one block of 256 threads, strided sums then a tree.
__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ p0, int n0,
                                                  const double *__restrict__ p1, int n1, double *c) {
    __shared__ double red[256];
    for (int which = 0; which < 2; which++) {
        const double *pp = which ? p1 : p0;
        const int n = which ? n1 : n0;
        if (which == 1 && !pp) break;
        double s = 0.0;
        for (int k = threadIdx.x; k < n; k += 256) s += pp[k];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) c[which] = red[0];
        __syncthreads();
    }
}

// ------------------------------------------------------------------ backward
//
// drho_e = E'(rho_e) sum_ij <Kbar(i,j), K_e^0(i,j)>
//        = E'(rho_e) |det J| sum_ij <L(X_ij), G^T M_ij G>
//        = E'(rho_e) |det J| sum_ij sum_mn M_ij[m][n] (G L(X_ij) G^T)[m][n],
// X_ij the stored Kbar block of (cells[e][i], cells[e][j]); L is self-adjoint.
template <int DIM, int NEN, int PREC>
__global__ __launch_bounds__(256) void k_backward(BwdParams P) {
    using T = typename CT<PREC>::T;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= P.n_cells) return;
    const int64_t NC = P.n_cells;
    constexpr int D2 = DIM * DIM;
    T G[DIM][DIM];
#pragma unroll
    for (int m = 0; m < DIM; m++)
#pragma unroll
        for (int a = 0; a < DIM; a++) G[m][a] = (T)P.geo[(int64_t)(m * DIM + a) * NC + e];
    const double det = P.geo[(int64_t)D2 * NC + e];
    int node[NEN], base[NEN], rowlen[NEN];
#pragma unroll
    for (int i = 0; i < NEN; i++) {
        node[i] = P.cells[e * NEN + i];
        base[i] = P.row_ptr[DIM * node[i]];
        rowlen[i] = P.row_ptr[DIM * node[i] + 1] - base[i];
    }
    const T lam = (T)P.lam, mu = (T)P.mu;
    double acc = 0.0;
    for (int i = 0; i < NEN; i++) {
        for (int j = 0; j < NEN; j++) {
            const int p = P.pos[(e * NEN + i) * NEN + j];
            T X[DIM][DIM];
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int b = 0; b < DIM; b++) {
                    double x = P.Kbar[base[i] + a * rowlen[i] + DIM * p + b];
                    if (P.mask && (P.mask[DIM * node[i] + a] | P.mask[DIM * node[j] + b])) x = 0.0;
                    X[a][b] = (T)x;
                }
            T tr = 0;
#pragma unroll
            for (int a = 0; a < DIM; a++) tr += X[a][a];
            T Y[DIM][DIM];
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int b = 0; b < DIM; b++) Y[a][b] = lam * X[a][b] + mu * X[b][a] + (a == b ? mu * tr : T(0));
            T GY[DIM][DIM];
#pragma unroll
            for (int m = 0; m < DIM; m++)
#pragma unroll
                for (int b = 0; b < DIM; b++) {
                    T t = 0;
#pragma unroll
                    for (int a = 0; a < DIM; a++) t += G[m][a] * Y[a][b];
                    GY[m][b] = t;
                }
            T blk = 0;
#pragma unroll
            for (int m = 0; m < DIM; m++)
#pragma unroll
                for (int n = 0; n < DIM; n++) {
                    T z = 0;
#pragma unroll
                    for (int b = 0; b < DIM; b++) z += GY[m][b] * G[n][b];
                    const T Mv = PREC == kF64 ? (T)P.M[(i * NEN + j) * D2 + m * DIM + n]
                                              : (T)P.M32[(i * NEN + j) * D2 + m * DIM + n];
                    blk += Mv * z;
                }
            acc += (double)blk;
        }
    }
    const double r = load_rho<PREC>(P.rho, e);
    const double dE = P.p * simp_pow(r, P.p - 1.0, P.ip >= 1 ? P.ip - 1 : -1) * (P.E0 - P.Emin);
    store_out<PREC>(P.drho, e, dE * det * acc);
}

// ---------------------------------------------------------------- launchers

template <int DIM, int NEN, int PREC>
static hipError_t launch_assemble_t(const AsmParams &P, int64_t ngroups, size_t lds, hipStream_t st) {
    if (ngroups <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_assemble<DIM, NEN, PREC>), dim3((unsigned)ngroups), dim3(256), lds, st, P);
    return hipGetLastError();
}

hipError_t launch_assemble(int elem, int prec, const AsmParams &P, int64_t ngroups, hipStream_t st) {
    const int dim = elem_dim(elem);
    const size_t csz = prec == kF64 ? 8 : 4;
    const size_t lds = csz * dim * dim * P.emax + 4 * (size_t)P.emax + 2 * (size_t)P.kmax * 64;
#define SOPTX_ASM(E, D, N)                                                         \
    case E:                                                                        \
        if (prec == kF64) return launch_assemble_t<D, N, kF64>(P, ngroups, lds, st); \
        if (prec == kF32) return launch_assemble_t<D, N, kF32>(P, ngroups, lds, st); \
        return launch_assemble_t<D, N, kBF16>(P, ngroups, lds, st);
    switch (elem) {
        SOPTX_ASM(SOPTX_QUAD4, 2, 4)
        SOPTX_ASM(SOPTX_TRI3, 2, 3)
        SOPTX_ASM(SOPTX_HEX8, 3, 8)
        SOPTX_ASM(SOPTX_TET10, 3, 10)
    default:
        return hipErrorInvalidValue;
    }
#undef SOPTX_ASM
}

template <int DIM, int NEN, int NQ, int PREC>
static hipError_t launch_energy_t(const EnergyParams &P, hipStream_t st) {
    const unsigned nb = (unsigned)((P.n_cells + 255) / 256);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL((k_energy<DIM, NEN, NQ, PREC>), dim3(nb), dim3(256), 0, st, P);
    return hipGetLastError();
}

hipError_t launch_energy(int elem, int prec, const EnergyParams &P, hipStream_t st) {
    const int pr = prec == kF64 ? kF64 : kF32;  // bf16 form evaluates energies in FP32
#define SOPTX_EN(E, D, N, Q)                                               \
    case E:                                                                \
        if (pr == kF64) return launch_energy_t<D, N, Q, kF64>(P, st);      \
        return launch_energy_t<D, N, Q, kF32>(P, st);
    switch (elem) {
        SOPTX_EN(SOPTX_QUAD4, 2, 4, 4)
        SOPTX_EN(SOPTX_TRI3, 2, 3, 1)
        SOPTX_EN(SOPTX_HEX8, 3, 8, 8)
        SOPTX_EN(SOPTX_TET10, 3, 10, 4)
    default:
        return hipErrorInvalidValue;
    }
#undef SOPTX_EN
}

hipError_t launch_dot_partials(const double *f, const double *u, int64_t n, double *partials, int nblocks,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_dot_partials, dim3(nblocks), dim3(256), 0, st, f, u, n, partials);
    return hipGetLastError();
}

hipError_t launch_finalize(const double *p0, int n0, const double *p1, int n1, double *c, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, p0, n0, p1, n1, c);
    return hipGetLastError();
}

template <int DIM, int NEN, int PREC>
static hipError_t launch_backward_t(const BwdParams &P, hipStream_t st) {
    const unsigned nb = (unsigned)((P.n_cells + 255) / 256);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL((k_backward<DIM, NEN, PREC>), dim3(nb), dim3(256), 0, st, P);
    return hipGetLastError();
}

hipError_t launch_backward(int elem, int prec, const BwdParams &P, hipStream_t st) {
    const int pr = prec == kF64 ? kF64 : kF32;
#define SOPTX_BW(E, D, N)                                          \
    case E:                                                        \
        if (pr == kF64) return launch_backward_t<D, N, kF64>(P, st); \
        return launch_backward_t<D, N, kF32>(P, st);
    switch (elem) {
        SOPTX_BW(SOPTX_QUAD4, 2, 4)
        SOPTX_BW(SOPTX_TRI3, 2, 3)
        SOPTX_BW(SOPTX_HEX8, 3, 8)
        SOPTX_BW(SOPTX_TET10, 3, 10)
    default:
        return hipErrorInvalidValue;
    }
#undef SOPTX_BW
}

}  // namespace soptx
