// gfx950 kernels of the equilibrium solve K u = f (arXiv 2505.02438,
// Sec. 2.2): a block-structured sparse product over the assembled CSR
// values and conjugate gradients preconditioned by the nodes' diagonal blocks (the iterative solver
// of the solver module, Sec. 3.2).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "block_sum.h"
#include "internal.h"
#include "kernels.h"

namespace soptx {

namespace {

// ------------------------------------------------------- solve (CG)
//
// The equilibrium system K u = f of the compliance problem, solved by
// conjugate gradients with a node-block Jacobi preconditioner on the assembled CSR values.
//
// y = K x.  K is a sum of DIM x DIM blocks, so a node's DIM rows share one
// neighbour list: row DIM I + a holds, for neighbour J = nb(I)[q], the
// entries of columns DIM J .. DIM J + DIM - 1 at row_ptr[DIM I + a] + DIM q.
// The kernel reads the neighbour lists (one id per block) instead of the
// column indices.  L lanes per node; lane s takes q = s, s + L, ...; the L
// partial sums of a row are added by an xor tree (a fixed order).  With
// xy_part, also the block partial of sum_r x_r y_r.
template <int DIM, int L>
__global__ __launch_bounds__(256) void k_spmv(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ nb,
                                              const double *__restrict__ K, const double *__restrict__ x,
                                              double *__restrict__ y, double *__restrict__ xy_part,
                                              int64_t n_nodes) {
    __shared__ double red[256];
    const int sub = threadIdx.x % L;
    const int64_t I = ((int64_t)blockIdx.x * 256 + threadIdx.x) / L;
    double acc[DIM];
#pragma unroll
    for (int a = 0; a < DIM; a++) acc[a] = 0.0;
    if (I < n_nodes) {
        const int b = row_ptr[DIM * I];
        const int rl = row_ptr[DIM * I + 1] - b;
        const int deg = rl / DIM;
        const int nbo = b / (DIM * DIM);
        for (int q = sub; q < deg; q += L) {
            const int J = nb[nbo + q];
            double xj[DIM];
#pragma unroll
            for (int e = 0; e < DIM; e++) xj[e] = x[(int64_t)DIM * J + e];
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int e = 0; e < DIM; e++) acc[a] += K[b + a * rl + DIM * q + e] * xj[e];
        }
    }
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1)
#pragma unroll
        for (int a = 0; a < DIM; a++) acc[a] += __shfl_xor(acc[a], off);
    double xy = 0.0;
    if (I < n_nodes && sub == 0) {
#pragma unroll
        for (int a = 0; a < DIM; a++) {
            y[DIM * I + a] = acc[a];
            xy += x[DIM * I + a] * acc[a];
        }
    }
    if (!xy_part) return;
    const double bs = block_sum_256(xy, red);
    if (threadIdx.x == 0) xy_part[blockIdx.x] = bs;
}

// Node-block Jacobi preconditioner: binv[I] = the inverse of node I's
// DIM x DIM diagonal block of K (row-major), by the adjugate.  A singular
// block (an isolated node) gives the inverse of its diagonal, 0 where that
// is 0, so such dofs stay put.
template <int DIM>
__global__ __launch_bounds__(256) void k_block_inv(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ nb,
                                                   const double *__restrict__ K, double *__restrict__ binv,
                                                   int64_t n_nodes) {
    const int64_t I = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (I >= n_nodes) return;
    const int b0 = row_ptr[DIM * I];
    const int rl = row_ptr[DIM * I + 1] - b0;
    const int nbo = b0 / (DIM * DIM);
    double B[DIM][DIM];
#pragma unroll
    for (int a = 0; a < DIM; a++)
#pragma unroll
        for (int c = 0; c < DIM; c++) B[a][c] = 0.0;
    for (int q = 0; q < rl / DIM; q++)
        if (nb[nbo + q] == I) {
#pragma unroll
            for (int a = 0; a < DIM; a++)
#pragma unroll
                for (int c = 0; c < DIM; c++) B[a][c] = K[b0 + a * rl + DIM * q + c];
        }
    double X[DIM][DIM];
    double det;
    if (DIM == 2) {
        det = B[0][0] * B[1][1] - B[0][1] * B[1][0];
        X[0][0] = B[1][1];
        X[0][1] = -B[0][1];
        X[1][0] = -B[1][0];
        X[1][1] = B[0][0];
    } else {
        X[0][0] = B[1][1] * B[2][2] - B[1][2] * B[2][1];
        X[0][1] = B[0][2] * B[2][1] - B[0][1] * B[2][2];
        X[0][2] = B[0][1] * B[1][2] - B[0][2] * B[1][1];
        X[1][0] = B[1][2] * B[2][0] - B[1][0] * B[2][2];
        X[1][1] = B[0][0] * B[2][2] - B[0][2] * B[2][0];
        X[1][2] = B[0][2] * B[1][0] - B[0][0] * B[1][2];
        X[2][0] = B[1][0] * B[2][1] - B[1][1] * B[2][0];
        X[2][1] = B[0][1] * B[2][0] - B[0][0] * B[2][1];
        X[2][2] = B[0][0] * B[1][1] - B[0][1] * B[1][0];
        det = B[0][0] * X[0][0] + B[0][1] * X[1][0] + B[0][2] * X[2][0];
    }
    double *o = binv + (int64_t)DIM * DIM * I;
    if (det != 0.0 && det == det) {
        const double id = 1.0 / det;
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int c = 0; c < DIM; c++) o[a * DIM + c] = X[a][c] * id;
    } else {
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int c = 0; c < DIM; c++) o[a * DIM + c] = (a == c && B[a][a] != 0.0) ? 1.0 / B[a][a] : 0.0;
    }
}

// One node's CG vector step (mode 0: r = f - q, p = z; mode 1: u += al p,
// r -= al q), then z = B^-1 r and the node's terms of r.z and r.r in dof order.
template <int DIM>
__device__ __forceinline__ void cg_node(int mode, double al, int64_t I, const double *__restrict__ f,
                                        double *__restrict__ u, double *__restrict__ r, double *__restrict__ z,
                                        double *__restrict__ p, const double *__restrict__ q,
                                        const double *__restrict__ binv, double &rz, double &rr) {
    const int64_t d0 = DIM * I;
    double ri[DIM];
    if (mode == 0) {
#pragma unroll
        for (int a = 0; a < DIM; a++) ri[a] = f[d0 + a] - q[d0 + a];
    } else {
#pragma unroll
        for (int a = 0; a < DIM; a++) {
            u[d0 + a] += al * p[d0 + a];
            ri[a] = r[d0 + a] - al * q[d0 + a];
        }
    }
    const double *bi = binv + (int64_t)DIM * DIM * I;
#pragma unroll
    for (int a = 0; a < DIM; a++) {
        double t = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; c++) t += bi[a * DIM + c] * ri[c];
        r[d0 + a] = ri[a];
        z[d0 + a] = t;
        if (mode == 0) p[d0 + a] = t;
        rz += ri[a] * t;
        rr += ri[a] * ri[a];
    }
}

// CG vector steps, one thread per node (its DIM dofs, so that z = B^-1 r
// uses the node's updated residual), block partials in a fixed order.
// Scalars sc: [0] r.z, [1] alpha, [2] beta, [3] r.r, [4] r0.r0, [5] p.q.
// mode 0 (start, q = K u): r = f - q, z = B^-1 r, p = z.
// mode 1 (iteration, q = K p): u += alpha p, r -= alpha q, z = B^-1 r.
// Both leave block partials of r.z (part[b]) and r.r (part[nb + b]); mode 0
// also of f.f (part[2 nb + b]).
template <int DIM>
__global__ __launch_bounds__(256) void k_cg_vec(int mode, const double *__restrict__ f, double *__restrict__ u,
                                                double *__restrict__ r, double *__restrict__ z,
                                                double *__restrict__ p, const double *__restrict__ q,
                                                const double *__restrict__ binv, const double *__restrict__ sc,
                                                double *__restrict__ part, int64_t n_nodes) {
    __shared__ double red[256];
    const int64_t I = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double rz = 0.0, rr = 0.0, ff = 0.0;
    if (I < n_nodes) {
        cg_node<DIM>(mode, mode == 0 ? 0.0 : sc[1], I, f, u, r, z, p, q, binv, rz, rr);
        if (mode == 0)
#pragma unroll
            for (int a = 0; a < DIM; a++) ff += f[DIM * I + a] * f[DIM * I + a];
    }
    const double brz = block_sum_256(rz, red);
    const double brr = block_sum_256(rr, red);
    const double bff = mode == 0 ? block_sum_256(ff, red) : 0.0;
    if (threadIdx.x == 0) {
        part[blockIdx.x] = brz;
        part[gridDim.x + blockIdx.x] = brr;
        if (mode == 0) part[2 * gridDim.x + blockIdx.x] = bff;
    }
}

// p = z + beta p
__global__ __launch_bounds__(256) void k_cg_p(double *__restrict__ p, const double *__restrict__ z,
                                              const double *__restrict__ sc, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = z[i] + sc[2] * p[i];
}

// The sum of n block partials in the order of k_cg_scalars (1024 strided
// sums, then a halving tree), computed by one block of 256 threads: thread t
// holds the strided sums t, t + 256, t + 512 and t + 768, does the tree's
// first two levels itself and block_sum_256 the rest.  Every block that calls
// it gets the same bits.
__device__ __forceinline__ double sum_as_scalars(const double *__restrict__ part, int n, double *red) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int g = 0; g < 4; g++)
        for (int k = (int)threadIdx.x + 256 * g; k < n; k += 1024) v[g] += part[k];
    v[0] += v[2];
    v[1] += v[3];
    v[0] += v[1];
    return block_sum_256(v[0], red);
}

// Fused iteration step for small systems: every block first forms
// alpha = r.z / p.q from the SpMV's partials (as k_cg_scalars would), then
// does k_cg_vec's mode 1.  Scalars are double-buffered by iteration parity
// (slot sc + 8 par holds this iteration's r.z); partials of r.z, r.r go to
// part_out, a different array from the p.q partials every block is reading.
template <int DIM>
__global__ __launch_bounds__(256) void k_cg_vec_fused(double *__restrict__ u, double *__restrict__ r,
                                                      double *__restrict__ z, double *__restrict__ p,
                                                      const double *__restrict__ q, const double *__restrict__ binv,
                                                      const double *__restrict__ pq_part, int n_pq,
                                                      const double *__restrict__ sc, double *__restrict__ part_out,
                                                      int64_t n_nodes) {
    __shared__ double red[256];
    const double al = sc[0] / sum_as_scalars(pq_part, n_pq, red);
    const int64_t I = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (I < n_nodes) cg_node<DIM>(1, al, I, nullptr, u, r, z, p, q, binv, rz, rr);
    const double brz = block_sum_256(rz, red);
    const double brr = block_sum_256(rr, red);
    if (threadIdx.x == 0) {
        part_out[blockIdx.x] = brz;
        part_out[gridDim.x + blockIdx.x] = brr;
    }
}

// Fused p step: every block forms beta = new r.z / r.z from the partials and
// updates p; block 0 writes the next iteration's scalars (new r.z, r.r) into
// the other parity slot, which no block of this launch reads.
__global__ __launch_bounds__(256) void k_cg_p_fused(double *__restrict__ p, const double *__restrict__ z,
                                                    const double *__restrict__ part, int nb, const double *sc_cur,
                                                    double *sc_next, int64_t n) {
    __shared__ double red[256];
    const double rz = sum_as_scalars(part, nb, red);
    const double beta = rz / sc_cur[0];
    if (blockIdx.x == 0) {
        const double rr = sum_as_scalars(part + nb, nb, red);
        if (threadIdx.x == 0) {
            sc_next[0] = rz;
            sc_next[2] = beta;
            sc_next[3] = rr;
        }
    }
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = z[i] + beta * p[i];
}

// One block of kScalThreads: sums of n block partials, thread t taking
// k = t, t + kScalThreads, ... in order, then a fixed tree.
// what 0 (start):     r.z and r.r from part -> sc[0], sc[3], sc[4] = sc[3]
// what 3 (start):     f.f from part -> sc[6]
// what 1 (alpha):     p.q from part -> sc[5], sc[1] = sc[0] / p.q
// what 2 (beta):      r.z, r.r from part -> sc[2] = new r.z / sc[0], sc[0], sc[3]
constexpr int kScalThreads = 1024;
__global__ __launch_bounds__(kScalThreads) void k_cg_scalars(int what, const double *__restrict__ part, int n,
                                                             double *sc) {
    __shared__ double red[2][kScalThreads];
    double t0 = 0.0, t1 = 0.0;
    for (int k = threadIdx.x; k < n; k += kScalThreads) {
        t0 += part[k];
        if (what != 1 && what != 3) t1 += part[n + k];
    }
    red[0][threadIdx.x] = t0;
    red[1][threadIdx.x] = t1;
    __syncthreads();
    for (int st = kScalThreads / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            red[0][threadIdx.x] += red[0][threadIdx.x + st];
            red[1][threadIdx.x] += red[1][threadIdx.x + st];
        }
        __syncthreads();
    }
    t0 = red[0][0];
    t1 = red[1][0];
    if (threadIdx.x != 0) return;
    if (what == 3) {
        sc[6] = t0;
    } else if (what == 0) {
        sc[0] = t0;
        sc[3] = t1;
        sc[4] = t1;
    } else if (what == 1) {
        sc[5] = t0;
        sc[1] = sc[0] / t0;
    } else {
        sc[2] = t0 / sc[0];
        sc[0] = t0;
        sc[3] = t1;
    }
}

}  // namespace

// ---------------------------------------------------------------- launchers

int64_t spmv_blocks(int dim, int64_t n_nodes) {
    const int L = dim == 3 ? 16 : 8;
    return (n_nodes * L + 255) / 256;
}

hipError_t launch_spmv(int dim, const int32_t *row_ptr, const int32_t *nb, const double *K, const double *x,
                       double *y, double *xy_part, int64_t n_nodes, hipStream_t st) {
    const unsigned g = (unsigned)spmv_blocks(dim, n_nodes);
    if (g == 0) return hipSuccess;
    if (dim == 3) hipLaunchKernelGGL((k_spmv<3, 16>), dim3(g), dim3(256), 0, st, row_ptr, nb, K, x, y, xy_part, n_nodes);
    else hipLaunchKernelGGL((k_spmv<2, 8>), dim3(g), dim3(256), 0, st, row_ptr, nb, K, x, y, xy_part, n_nodes);
    return hipGetLastError();
}

int64_t cg_vec_blocks(int dim, int64_t ndof) { return (ndof / dim + 255) / 256; }

hipError_t launch_block_inv(int dim, const int32_t *row_ptr, const int32_t *nb, const double *K, double *binv,
                            int64_t n_nodes, hipStream_t st) {
    const unsigned g = (unsigned)((n_nodes + 255) / 256);
    if (g == 0) return hipSuccess;
    if (dim == 3) hipLaunchKernelGGL(k_block_inv<3>, dim3(g), dim3(256), 0, st, row_ptr, nb, K, binv, n_nodes);
    else hipLaunchKernelGGL(k_block_inv<2>, dim3(g), dim3(256), 0, st, row_ptr, nb, K, binv, n_nodes);
    return hipGetLastError();
}

hipError_t launch_cg_vec(int dim, int mode, const double *f, double *u, double *r, double *z, double *p,
                         const double *q, const double *binv, const double *sc, double *part, int64_t ndof,
                         hipStream_t st) {
    const unsigned g = (unsigned)cg_vec_blocks(dim, ndof);
    if (g == 0) return hipSuccess;
    if (dim == 3)
        hipLaunchKernelGGL(k_cg_vec<3>, dim3(g), dim3(256), 0, st, mode, f, u, r, z, p, q, binv, sc, part, ndof / 3);
    else
        hipLaunchKernelGGL(k_cg_vec<2>, dim3(g), dim3(256), 0, st, mode, f, u, r, z, p, q, binv, sc, part, ndof / 2);
    return hipGetLastError();
}

hipError_t launch_cg_vec_fused(int dim, double *u, double *r, double *z, double *p, const double *q,
                               const double *binv, const double *pq_part, int n_pq, const double *sc,
                               double *part_out, int64_t ndof, hipStream_t st) {
    const unsigned g = (unsigned)cg_vec_blocks(dim, ndof);
    if (g == 0) return hipSuccess;
    if (dim == 3)
        hipLaunchKernelGGL(k_cg_vec_fused<3>, dim3(g), dim3(256), 0, st, u, r, z, p, q, binv, pq_part, n_pq, sc,
                           part_out, ndof / 3);
    else
        hipLaunchKernelGGL(k_cg_vec_fused<2>, dim3(g), dim3(256), 0, st, u, r, z, p, q, binv, pq_part, n_pq, sc,
                           part_out, ndof / 2);
    return hipGetLastError();
}

hipError_t launch_cg_p_fused(double *p, const double *z, const double *part, int nb, const double *sc_cur,
                             double *sc_next, int64_t n, hipStream_t st) {
    const int64_t g0 = (n + 255) / 256;
    const unsigned g = (unsigned)(g0 < 1024 ? g0 : 1024);
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cg_p_fused, dim3(g), dim3(256), 0, st, p, z, part, nb, sc_cur, sc_next, n);
    return hipGetLastError();
}

hipError_t launch_cg_p(double *p, const double *z, const double *sc, int64_t n, hipStream_t st) {
    const unsigned g = (unsigned)((n + 255) / 256);
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cg_p, dim3(g), dim3(256), 0, st, p, z, sc, n);
    return hipGetLastError();
}

hipError_t launch_cg_scalars(int what, const double *part, int n, double *sc, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(kScalThreads), 0, st, what, part, n, sc);
    return hipGetLastError();
}

}  // namespace soptx
