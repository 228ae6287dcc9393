// gfx950 kernels of the filter step (arXiv 2505.02438, Sec. 2.4): products
// with the filter matrix H for the sensitivity filter, the density filter
// (with the Heaviside projection fused into its output) and the density
// filter's chain rule.
//
// H is CSR (int32 columns, FP64 weights, separate arrays).  L lanes take one
// row: lane s reads entries s, s + L, ... of the row (L consecutive entries
// per step, so the column and weight loads are contiguous), gathers the
// neighbour values (small vectors, resident in L2 / MALL) and the L partial
// sums are added by an xor tree, a fixed order.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "kernels.h"

namespace soptx {

namespace {

constexpr double kSensGamma = 1e-3;

// MODE 0: density filter      out0 = sum w v_j x_j / hsv_i; out1 = Heaviside(out0) if non-null
// MODE 1: chain rule product  out0 = v_i sum w x_j
// MODE 2: sensitivity filter  out0 = sum w x_j y_j / (max(gamma, x_i) hs_i)
template <int L, int MODE>
__global__ __launch_bounds__(256) void k_filter(FilterArgs F, const double *__restrict__ x,
                                                const double *__restrict__ y, double beta,
                                                double *__restrict__ out0, double *__restrict__ out1) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t i = t / L;
    const int s = (int)(t % L);
    const bool live = i < F.n;
    double acc = 0.0;
    if (live) {
        const int32_t beg = F.row_ptr[i], end = F.row_ptr[i + 1];
        for (int32_t k = beg + s; k < end; k += L) {
            const int32_t j = F.col[k];
            const double w = F.w[k];
            if (MODE == 0) acc += w * (F.v[j] * x[j]);
            else if (MODE == 1) acc += w * x[j];
            else acc += w * (x[j] * y[j]);
        }
    }
#pragma unroll
    for (int m = L / 2; m > 0; m >>= 1) acc += __shfl_xor(acc, m, L);
    if (!live || s != 0) return;
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
hipError_t launch_mode(const FilterArgs &F, int lanes, const double *x, const double *y, double beta, double *o0,
                       double *o1, hipStream_t st) {
    if (F.n <= 0) return hipSuccess;
    const unsigned g = (unsigned)((F.n * lanes + 255) / 256);
    switch (lanes) {
    case 4: hipLaunchKernelGGL((k_filter<4, MODE>), dim3(g), dim3(256), 0, st, F, x, y, beta, o0, o1); break;
    case 8: hipLaunchKernelGGL((k_filter<8, MODE>), dim3(g), dim3(256), 0, st, F, x, y, beta, o0, o1); break;
    case 16: hipLaunchKernelGGL((k_filter<16, MODE>), dim3(g), dim3(256), 0, st, F, x, y, beta, o0, o1); break;
    case 32: hipLaunchKernelGGL((k_filter<32, MODE>), dim3(g), dim3(256), 0, st, F, x, y, beta, o0, o1); break;
    case 64: hipLaunchKernelGGL((k_filter<64, MODE>), dim3(g), dim3(256), 0, st, F, x, y, beta, o0, o1); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_filter_density(const FilterArgs &F, int lanes, const double *rho, double beta, double *rho_tilde,
                                 double *rho_bar, hipStream_t st) {
    return launch_mode<0>(F, lanes, rho, nullptr, beta, rho_tilde, rho_bar, st);
}

hipError_t launch_filter_sensitivity(const FilterArgs &F, int lanes, const double *rho, const double *dc,
                                     double *dc_out, hipStream_t st) {
    return launch_mode<2>(F, lanes, rho, dc, 0.0, dc_out, nullptr, st);
}

hipError_t launch_filter_backward(const FilterArgs &F, int lanes, const double *rho_tilde, double beta,
                                  const double *g, double *tmp, double *grad, hipStream_t st) {
    if (F.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_filter_scale, dim3((unsigned)((F.n + 255) / 256)), dim3(256), 0, st, g, rho_tilde, beta,
                       F.hsv, tmp, F.n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_mode<1>(F, lanes, tmp, nullptr, 0.0, grad, nullptr, st);
}

}  // namespace soptx
