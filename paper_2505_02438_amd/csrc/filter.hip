// gfx950 kernels of the filter step (arXiv 2505.02438, Sec. 2.4): products
// with the filter matrix H for the sensitivity filter, the density filter
// (with the Heaviside projection fused into its output) and the density
// filter's chain rule.
//
// H is CSR (int32 columns, FP64 weights, separate arrays).  A block takes R
// consecutive rows, whose entries are contiguous in the CSR arrays: its 256
// threads stream them in chunks of kFilterChunk entries (fully coalesced
// column and weight loads, one gather of the neighbour values per entry, the
// small vectors staying in L2 / MALL) and store each product w * t to LDS;
// then thread r adds row r's products in ascending column order.  The sum of
// a row is therefore formed exactly as a sequential CSR product forms it:
// each product rounded, then added left to right from zero.  R <= 256; rows
// longer than a chunk carry their running sum across chunks.  Contraction is
// off in both product kernels, so they also agree on the fused Heaviside
// projection.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "kernels.h"

namespace soptx {

namespace {

constexpr double kSensGamma = 1e-3;

// MODE 0: density filter      out0 = sum w (v_j x_j) / hsv_i; out1 = Heaviside(out0) if non-null
// MODE 1: chain rule product  out0 = v_i sum w x_j
// MODE 2: sensitivity filter  out0 = sum w (x_j y_j) / (max(gamma, x_i) hs_i)
template <int MODE>
__global__ __launch_bounds__(256) void k_filter(FilterArgs F, int R, const double *__restrict__ x,
                                                const double *__restrict__ y, double beta,
                                                double *__restrict__ out0, double *__restrict__ out1) {
#pragma clang fp contract(off)
    __shared__ double prod[kFilterChunk];
    const int64_t r0 = (int64_t)blockIdx.x * R;
    const int64_t r1 = r0 + R < F.n ? r0 + R : F.n;
    const int32_t e0 = F.row_ptr[r0], e1 = F.row_ptr[r1];
    const int64_t i = r0 + threadIdx.x;  // this thread's row
    const bool owner = i < r1;
    const int32_t rb = owner ? F.row_ptr[i] : 0, re = owner ? F.row_ptr[i + 1] : 0;
    double acc = 0.0;
    for (int32_t c0 = e0; c0 < e1; c0 += kFilterChunk) {
        const int32_t c1 = c0 + kFilterChunk < e1 ? c0 + kFilterChunk : e1;
        for (int32_t k = c0 + (int32_t)threadIdx.x; k < c1; k += 256) {
            const int32_t j = F.col[k];
            double t;
            if (MODE == 0) t = F.v[j] * x[j];
            else if (MODE == 1) t = x[j];
            else t = x[j] * y[j];
            prod[k - c0] = F.w[k] * t;
        }
        __syncthreads();
        if (owner) {
            const int32_t b = rb > c0 ? rb : c0, e = re < c1 ? re : c1;
            for (int32_t k = b; k < e; k++) acc += prod[k - c0];
        }
        __syncthreads();
    }
    if (!owner) return;
    if (MODE == 0) {
        const double r = acc / F.hsv[i];
        out0[i] = r;
        if (out1) out1[i] = 1.0 - exp(-beta * r) + r * exp(-beta);
    } else if (MODE == 1) {
        out0[i] = F.v[i] * acc;
    } else {
        out0[i] = acc / (fmax(kSensGamma, x[i]) * F.hs[i]);
    }
}

// The same products when H is a stencil on a structured grid (numbered with
// the last axis fastest): one thread per row, the offsets in ascending linear
// order (= ascending column), those outside the grid skipped.  Contraction is
// off so that each product is rounded before it is added, as in the row-block
// kernel and a sequential CSR product.
template <int MODE>
__global__ __launch_bounds__(256) void k_filter_stencil(FilterArgs F, const double *__restrict__ x,
                                                        const double *__restrict__ y, double beta,
                                                        double *__restrict__ out0, double *__restrict__ out1) {
#pragma clang fp contract(off)
    const int i = (int)(blockIdx.x * 256 + threadIdx.x);  // n < 2^31 (int32 CSR)
    if (i >= F.n) return;
    const int N0 = (int)F.N[0], N1 = (int)F.N[1], N2 = (int)F.N[2];
    const int c2 = i % N2, q = i / N2;
    const int c1 = q % N1, c0 = q / N1;
    double acc = 0.0;
    // 8 offsets at a time: every gather issued first (an offset outside the
    // grid reads row i itself and is not added), then added in offset order
    constexpr int U = 8;
    for (int s0 = 0; s0 < F.S; s0 += U) {
        double t[U], w[U];
        bool in[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int s = s0 + u < F.S ? s0 + u : F.S - 1;
            const int a = c0 + F.sdel[3 * s], b = c1 + F.sdel[3 * s + 1], c = c2 + F.sdel[3 * s + 2];
            in[u] = s0 + u < F.S && a >= 0 && a < N0 && b >= 0 && b < N1 && c >= 0 && c < N2;
            const int j = in[u] ? (a * N1 + b) * N2 + c : i;
            w[u] = F.sw[s];
            if (MODE == 0) t[u] = F.v[j] * x[j];
            else if (MODE == 1) t[u] = x[j];
            else t[u] = x[j] * y[j];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const double p = w[u] * t[u];
            if (in[u]) acc = acc + p;
        }
    }
    if (MODE == 0) {
        const double r = acc / F.hsv[i];
        out0[i] = r;
        if (out1) out1[i] = 1.0 - exp(-beta * r) + r * exp(-beta);
    } else if (MODE == 1) {
        out0[i] = F.v[i] * acc;
    } else {
        out0[i] = acc / (fmax(kSensGamma, x[i]) * F.hs[i]);
    }
}

// t_i = g_i h'(rho~_i) / hsv_i with h' the Heaviside derivative (1 without
// rho~): the right-hand factor of the chain-rule product
__global__ __launch_bounds__(256) void k_filter_scale(const double *__restrict__ g, const double *__restrict__ rt,
                                                      double beta, const double *__restrict__ hsv,
                                                      double *__restrict__ t, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double gi = g[i];
    if (rt) gi = gi * (beta * exp(-beta * rt[i]) + exp(-beta));
    t[i] = gi / hsv[i];
}

template <int MODE>
hipError_t launch_mode(const FilterArgs &F, int R, const double *x, const double *y, double beta, double *o0,
                       double *o1, hipStream_t st) {
    if (F.n <= 0) return hipSuccess;
    if (F.S > 0) {
        hipLaunchKernelGGL(k_filter_stencil<MODE>, dim3((unsigned)((F.n + 255) / 256)), dim3(256), 0, st, F, x, y,
                           beta, o0, o1);
        return hipGetLastError();
    }
    if (R < 1 || R > 256) return hipErrorInvalidValue;
    const unsigned g = (unsigned)((F.n + R - 1) / R);
    hipLaunchKernelGGL(k_filter<MODE>, dim3(g), dim3(256), 0, st, F, R, x, y, beta, o0, o1);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_filter_density(const FilterArgs &F, int R, const double *rho, double beta, double *rho_tilde,
                                 double *rho_bar, hipStream_t st) {
    return launch_mode<0>(F, R, rho, nullptr, beta, rho_tilde, rho_bar, st);
}

hipError_t launch_filter_sensitivity(const FilterArgs &F, int R, const double *rho, const double *dc,
                                     double *dc_out, hipStream_t st) {
    return launch_mode<2>(F, R, rho, dc, 0.0, dc_out, nullptr, st);
}

hipError_t launch_filter_backward(const FilterArgs &F, int R, const double *rho_tilde, double beta,
                                  const double *g, double *tmp, double *grad, hipStream_t st) {
    if (F.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_filter_scale, dim3((unsigned)((F.n + 255) / 256)), dim3(256), 0, st, g, rho_tilde, beta,
                       F.hsv, tmp, F.n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_mode<1>(F, R, tmp, nullptr, 0.0, grad, nullptr, st);
}

}  // namespace soptx
