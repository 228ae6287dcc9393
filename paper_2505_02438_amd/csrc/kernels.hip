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

#include <algorithm>
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

// Reads of tables that no kernel writes (plan, reference tensor) through the
// constant address space: at wave-uniform indices they become scalar loads
// through the scalar cache, unaffected by the wave-level LDS fences.
template <class T>
__device__ __forceinline__ T ldc(const T *base, int64_t idx) {
    return ((const __attribute__((address_space(4))) T *)(base))[idx];
}
__device__ __forceinline__ double ref_f64(const double *base, int idx) { return ldc(base, idx); }
__device__ __forceinline__ float ref_f32(const float *base, int idx) { return ldc(base, idx); }

}  // namespace

// ------------------------------------------------------------------ assembly
//
// acc += G'^T M_ij G' in the precision of the form (FP64 accumulation)
template <int DIM, int PREC, typename T>
__device__ __forceinline__ void accumulate(const T (&G)[DIM][DIM], const T (&M)[DIM * DIM], double (&acc)[DIM][DIM]) {
    if (PREC == kBF16) {
        // bf16 inputs, fp32 accumulation: A[a][b] = sum_mn M[m][n] W[m,a][n,b]
        // with both GEMM operands rounded to bf16, W = G'[m][a] G'[n][b]
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int b = 0; b < DIM; b++) {
                float s = 0.0f;
#pragma unroll
                for (int m = 0; m < DIM; m++)
#pragma unroll
                    for (int n = 0; n < DIM; n++)
                        s += (float)M[m * DIM + n] * bf16_round((float)G[m][a] * (float)G[n][b]);
                acc[a][b] += (double)s;
            }
        return;
    }
    T Tm[DIM][DIM];
#pragma unroll
    for (int m = 0; m < DIM; m++)
#pragma unroll
        for (int b = 0; b < DIM; b++) {
            T s = 0;
#pragma unroll
            for (int n = 0; n < DIM; n++) s += M[m * DIM + n] * G[n][b];
            Tm[m][b] = s;
        }
    if (PREC == kF64) {
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int b = 0; b < DIM; b++)
#pragma unroll
                for (int m = 0; m < DIM; m++) acc[a][b] += (double)G[m][a] * (double)Tm[m][b];
    } else {
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int b = 0; b < DIM; b++) {
                T s = 0;
#pragma unroll
                for (int m = 0; m < DIM; m++) s += G[m][a] * Tm[m][b];
                acc[a][b] += (double)s;
            }
    }
}

// G' of the element in LDS slot `slot` and the reference block M_ij
template <int DIM, int NEN, int PREC, typename T>
__device__ __forceinline__ void fetch_contrib(const AsmParams &P, const T *sG, int slot, int pk, T (&G)[DIM][DIM],
                                              T (&M)[DIM * DIM]) {
    constexpr int D2 = DIM * DIM;
    const int i = (pk >> 8) & 255, j = pk & 255;
#pragma unroll
    for (int m = 0; m < DIM; m++)
#pragma unroll
        for (int a = 0; a < DIM; a++) G[m][a] = sG[(m * DIM + a) * kGroupElems + slot];
    const int mij = (i * NEN + j) * D2;
#pragma unroll
    for (int x = 0; x < D2; x++) {
        if (PREC == kF64) M[x] = (T)ref_f64(P.M, mij + x);
        else if (PREC == kF32) M[x] = (T)ref_f32(P.M32, mij + x);
        else M[x] = (T)ref_f32(P.Mbf, mij + x);
    }
}

size_t assemble_lds_bytes(int dim, int prec, int64_t stage, int kmax) {
    const size_t csz = prec == kF64 ? 8 : 4;
    return 8 * (size_t)stage + csz * dim * dim * kGroupElems + 64 * 2 * 4 + 2 * (size_t)kmax * 64;
}

// Persistent assembly.  One workgroup of 8 waves per CU walks the node groups
// blockIdx.x, blockIdx.x + gridDim.x, ...  For a group (up to 64 nodes with
// one connectivity signature):
//   1. its elements' G' = sqrt(E(rho) det J) J^-1 are staged in LDS (the data
//      was loaded to registers while the previous group was assembled);
//   2. waves take neighbour positions from a ticket; lane l = node l of the
//      group walks the position's contributions (the same (k, i, j) on every
//      lane, so M_ij comes through scalar loads) and writes its finished
//      DIM x DIM block into the group's row blocks in LDS;
//   3. every node's DIM rows (contiguous in CSR) are written out as one
//      contiguous run; the stores drain while the next group is assembled.
// Summation order of a stored block: the signature's contribution order
// (ascending element within the block), then L(A) = lam A + mu A^T +
// mu tr(A) I; fixed by the mesh, independent of waves and streams.
constexpr int kAsmThreads = 1024;  // 16 waves share one group's LDS

template <int DIM, int NEN, int PREC>
__global__ __launch_bounds__(kAsmThreads, 1) void k_assemble(AsmParams P) {
    using T = typename CT<PREC>::T;
    constexpr int D2 = DIM * DIM;
    constexpr int NT = kAsmThreads;
    constexpr int NPF = (kMaxAdjacent * 64 + NT - 1) / NT;  // slot-table entries prefetched per thread
    extern __shared__ __align__(16) unsigned char smem[];
    double *stage = reinterpret_cast<double *>(smem);                           // [P.stage]
    T *sG = reinterpret_cast<T *>(stage + P.stage);                              // [D2][kGroupElems]
    int32_t *srows = reinterpret_cast<int32_t *>(sG + D2 * kGroupElems);         // [64][2]
    uint16_t *sn2l = reinterpret_cast<uint16_t *>(srows + 128);                  // [kmax][64]
    __shared__ int ticket;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = wave_uniform(tid >> 6);
    const int64_t NC = P.n_cells;

    int g = blockIdx.x;
    if (g >= P.n_groups) return;

    // next group, prefetched to registers: one element per thread (geometry and
    // density), the slot table and the row offsets
    int pid;
    double pd[D2 + 2];
    int pn2l[NPF];
    int prow;
    auto load_ids = [&](int gg) {
        const int eoff = ldc(P.grp_info, 5 * gg + 2);
        const int ne = ldc(P.grp_info, 5 * gg + 3);
        pid = tid < ne ? P.grp_elems[eoff + tid] : -1;
        const int sg = ldc(P.grp_info, 5 * gg + 0);
        const int off = ldc(P.grp_info, 5 * gg + 4);
        const int nk = ldc(P.sig_info, 4 * sg + 0) * 64;
#pragma unroll
        for (int r = 0; r < NPF; r++) pn2l[r] = tid + r * NT < nk ? P.grp_n2l[off + tid + r * NT] : 0;
        prow = tid < 128 ? P.grp_rows[(int64_t)gg * 128 + tid] : 0;
    };
    auto load_data = [&]() {
        if (pid >= 0) {
#pragma unroll
            for (int c = 0; c <= D2; c++) pd[c] = P.geo[(int64_t)c * NC + pid];
            pd[D2 + 1] = load_rho<PREC>(P.rho, pid);
        }
    };
    auto write_group = [&](int gg) {
        if (pid >= 0) {
            const double E = P.Emin + simp_pow(pd[D2 + 1], P.p, P.ip) * (P.E0 - P.Emin);
            const double q = sqrt(E * pd[D2]);
#pragma unroll
            for (int c = 0; c < D2; c++) sG[c * kGroupElems + tid] = (T)(q * pd[c]);
        }
        const int sg = ldc(P.grp_info, 5 * gg + 0);
        const int nk = ldc(P.sig_info, 4 * sg + 0) * 64;
#pragma unroll
        for (int r = 0; r < NPF; r++)
            if (tid + r * NT < nk) sn2l[tid + r * NT] = (uint16_t)pn2l[r];
        if (tid < 128) srows[tid] = prow;
        if (tid == 0) ticket = 0;
    };

    load_ids(g);
    load_data();
    write_group(g);
    int gn = g + gridDim.x;
    if (gn < P.n_groups) load_ids(gn);
    // workgroups alternate between a compute phase and a store phase; odd
    // ones start half a period late so that the device's stores are spread
    // over time instead of arriving in waves
    if (blockIdx.x & 1) {
        for (int k = 0; k < P.desync; k++) __builtin_amdgcn_s_sleep(127);
    }

    for (;;) {
        __syncthreads();  // LDS of group g complete; stage free
        if (gn < P.n_groups) load_data();  // in flight while group g is assembled
        const int sig = ldc(P.grp_info, 5 * g + 0);
        const int nn = ldc(P.grp_info, 5 * g + 1);
        const int deg = ldc(P.sig_info, 4 * sig + 1);
        const int posoff = ldc(P.sig_info, 4 * sig + 2);
        const int blk = ldc(P.sig_info, 4 * sig + 3);
        const int rl = DIM * deg;  // row length
        const bool active = lane < nn;
        double *mystage = stage + lane * blk;

        for (;;) {
            int r = 0;
            if (lane == 0) r = atomicAdd(&ticket, 1);
            r = wave_uniform(r);
            if (r >= deg) break;
            const int p = ldc(P.sig_order, posoff + r);
            const int c0 = ldc(P.sig_pos_ptr, posoff + p), c1 = ldc(P.sig_pos_ptr, posoff + p + 1);
            double acc[DIM][DIM];
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int b = 0; b < DIM; b++) acc[a][b] = 0.0;
            for (int t = c0; t < c1; t += 2) {
                // two contributions per round trip
                const int pk0 = ldc(P.sig_contrib, t);
                const bool two = t + 1 < c1;
                const int pk1 = two ? ldc(P.sig_contrib, t + 1) : pk0;
                const int s0 = sn2l[(pk0 >> 16) * 64 + lane];
                const int s1 = sn2l[(pk1 >> 16) * 64 + lane];
                T G0[DIM][DIM], G1[DIM][DIM], M0[D2], M1[D2];
                fetch_contrib<DIM, NEN, PREC>(P, sG, s0, pk0, G0, M0);
                fetch_contrib<DIM, NEN, PREC>(P, sG, s1, pk1, G1, M1);
                accumulate<DIM, PREC>(G0, M0, acc);
                if (two) accumulate<DIM, PREC>(G1, M1, acc);
            }
            double tr = 0.0;
#pragma unroll
            for (int a = 0; a < DIM; a++) tr += acc[a][a];
            if (active) {
#pragma unroll
                for (int a = 0; a < DIM; a++)
#pragma unroll
                    for (int b = 0; b < DIM; b++) {
                        double o = P.lam * acc[a][b] + P.mu * acc[b][a];
                        if (a == b) o += P.mu * tr;
                        mystage[a * rl + DIM * p + b] = o;
                    }
            }
        }
        __syncthreads();  // all row blocks of the group staged
        // node n's DIM rows are contiguous in CSR: one run of DIM * rl values
        const int bsz = DIM * rl;
        for (int n = w; n < nn; n += NT / 64) {
            const int base = srows[2 * n];
            const double *src = stage + n * blk;
            for (int o = lane; o < bsz; o += 64) P.K[base + o] = src[o];
        }
        __syncthreads();  // every stage value has been read
        if (gn >= P.n_groups) break;
        g = gn;
        write_group(g);
        gn = g + gridDim.x;
        if (gn < P.n_groups) load_ids(gn);
    }
}

// Dirichlet rows and columns (zero prescribed values): for every fixed dof r,
// K[r,:] = 0, K[:,r] = 0, K[r,r] = 1, pattern unchanged.  Runs after the
// assembly on the same stream.  16 lanes per node; entry (c, r) of a fixed
// column is found by binary search in row c (the pattern is symmetric).
template <int DIM>
__global__ __launch_bounds__(256) void k_dirichlet(const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col_idx,
                                                   const uint8_t *__restrict__ mask, double *K,
                                                   int64_t n_nodes) {
    const int64_t I = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    const int l = threadIdx.x & 15;
    if (I >= n_nodes) return;
    for (int a = 0; a < DIM; a++) {
        const int r = (int)(DIM * I + a);
        if (!mask[r]) continue;
        const int b0 = row_ptr[r], b1 = row_ptr[r + 1];
        for (int k = b0 + l; k < b1; k += 16) {
            const int c = col_idx[k];
            K[k] = (c == r) ? 1.0 : 0.0;
            // entry (c, r)
            int lo = row_ptr[c], hi = row_ptr[c + 1] - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (col_idx[mid] < r) lo = mid + 1; else hi = mid;
            }
            K[lo] = (c == r) ? 1.0 : 0.0;
        }
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
static hipError_t launch_assemble_t(const AsmParams &P, int64_t ngroups, hipStream_t st) {
    if (ngroups <= 0) return hipSuccess;
    const size_t lds = assemble_lds_bytes(DIM, PREC, P.stage, P.kmax);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const void *fn = reinterpret_cast<const void *>(&k_assemble<DIM, NEN, PREC>);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kAsmThreads, lds);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    const int ncu = P.n_cu > 0 ? P.n_cu : 256;
    const int64_t grid = std::min<int64_t>(ngroups, (int64_t)per_cu * ncu);
    hipLaunchKernelGGL((k_assemble<DIM, NEN, PREC>), dim3((unsigned)grid), dim3(kAsmThreads), lds, st, P);
    return hipGetLastError();
}

hipError_t launch_assemble(int elem, int prec, const AsmParams &P, int64_t ngroups, hipStream_t st) {
#define SOPTX_ASM(E, D, N)                                                    \
    case E:                                                                   \
        if (prec == kF64) return launch_assemble_t<D, N, kF64>(P, ngroups, st); \
        if (prec == kF32) return launch_assemble_t<D, N, kF32>(P, ngroups, st); \
        return launch_assemble_t<D, N, kBF16>(P, ngroups, st);
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

hipError_t launch_dirichlet(int dim, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *mask,
                            double *K, int64_t n_nodes, hipStream_t st) {
    const unsigned nb = (unsigned)((n_nodes + 15) / 16);
    if (nb == 0) return hipSuccess;
    if (dim == 2) hipLaunchKernelGGL(k_dirichlet<2>, dim3(nb), dim3(256), 0, st, row_ptr, col_idx, mask, K, n_nodes);
    else hipLaunchKernelGGL(k_dirichlet<3>, dim3(nb), dim3(256), 0, st, row_ptr, col_idx, mask, K, n_nodes);
    return hipGetLastError();
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
