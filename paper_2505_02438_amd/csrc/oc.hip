// gfx950 kernels of the optimality-criteria update (arXiv 2505.02438,
// Sec. 2.3, Algorithm 1): the clamped, damped update of the design variables
// and the bisection on the multiplier lambda of the volume constraint.
//
// Bisection on the device.  A pass of k_oc_eval evaluates vol at the 15 nodes
// of the depth-4 tree of midpoints that the next 4 steps of the sequential
// loop can reach from the current bracket (l1, l2): node 0 is (l1 + l2) / 2,
// the child taken when vol > V* (l1 = mid) is 2k + 1, the other child
// (l2 = mid) is 2k + 2, each midpoint computed as the loop computes it.  Then
// k_oc_decide (one block) sums the block partials in a fixed order and walks
// the tree with the loop's test before every step, so it takes exactly the
// loop's decisions for this vol.  The state lives in device memory:
//   st[0] l1, st[1] l2, st[2] last mid, st[3] vol at it, st[4] steps,
//   st[5] done flag, st[6] max change.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "kernels.h"

namespace soptx {

namespace {

struct OcArgs {
    const double *rho, *dc, *dv;
    int64_t n;
    double move, eta;
};

// rho_new at lambda; comparisons written out so that a NaN propagates as it
// does through max / min of IEEE arithmetic with NaN operands
__device__ __forceinline__ double oc_new(double rho, double dc, double dv, double lam, double move, double eta) {
    const double num = -dc > 0.0 ? -dc : 0.0;
    const double B = num / (lam * dv);
    double be;
    if (eta == 0.5) be = sqrt(B);
    else if (eta == 1.0) be = B;
    else be = pow(B, eta);
    double c = rho * be;
    const double lo = rho - move > 0.0 ? rho - move : 0.0;
    const double hi = rho + move < 1.0 ? rho + move : 1.0;
    if (c < lo) c = lo;
    if (c > hi) c = hi;
    return c;
}

__device__ __forceinline__ void tree_mids(double l1, double l2, double (&lam)[kOcNodes]) {
    double a[kOcNodes], b[kOcNodes];
    a[0] = l1;
    b[0] = l2;
#pragma unroll
    for (int k = 0; k < kOcNodes; k++) {
        lam[k] = 0.5 * (a[k] + b[k]);
        if (2 * k + 2 < kOcNodes) {
            a[2 * k + 1] = lam[k];  // vol > V*: l1 = mid
            b[2 * k + 1] = b[k];
            a[2 * k + 2] = a[k];    // otherwise: l2 = mid
            b[2 * k + 2] = lam[k];
        }
    }
}

__global__ __launch_bounds__(256) void k_oc_init(double *st, double lmax) {
    if (threadIdx.x == 0) {
        st[0] = 0.0;
        st[1] = lmax;
        st[2] = 0.0;
        st[3] = 0.0;
        st[4] = 0.0;
        st[5] = 0.0;
        st[6] = 0.0;
    }
}

// sum over the 64 lanes of a wave by a fixed butterfly (every lane gets it)
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

// part[node * gridDim.x + block] = sum over the block's elements of dv rho_new(lambda_node):
// per thread in element order, then each wave by a butterfly, then the 4
// waves in order
__global__ __launch_bounds__(256) void k_oc_eval(OcArgs A, const double *__restrict__ st, double *__restrict__ part) {
    __shared__ double red[4][kOcNodes];
    if (st[5] != 0.0) return;  // uniform: the bisection has ended
    double lam[kOcNodes], acc[kOcNodes];
    tree_mids(st[0], st[1], lam);
#pragma unroll
    for (int k = 0; k < kOcNodes; k++) acc[k] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < A.n; e += (int64_t)gridDim.x * 256) {
        const double r = A.rho[e], d = A.dc[e], v = A.dv[e];
#pragma unroll
        for (int k = 0; k < kOcNodes; k++) acc[k] += v * oc_new(r, d, v, lam[k], A.move, A.eta);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kOcNodes; k++) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) red[w][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < kOcNodes) {
        const int k = threadIdx.x;
        part[(int64_t)k * gridDim.x + blockIdx.x] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
}

// one wave per tree node (kOcNodes <= 16 waves of the 1024-thread block):
// lane l sums blocks l, l + 64, ... in order, then a butterfly
static_assert(kOcNodes <= 16, "one wave per tree node in a 1024-thread block");
__global__ __launch_bounds__(1024) void k_oc_decide(const double *__restrict__ part, int nblk, double vol_target,
                                                    double tol, int max_steps, double *st) {
    __shared__ double vol[kOcNodes];
    if (st[5] != 0.0) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (w < kOcNodes) {
        double t = 0.0;
        for (int b = lane; b < nblk; b += 64) t += part[(int64_t)w * nblk + b];
        t = wave_sum(t);
        if (lane == 0) vol[w] = t;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double l1 = st[0], l2 = st[1], lam = st[2], vl = st[3];
    int steps = (int)st[4];
    int node = 0;
    for (int level = 0; level < kOcDepth; level++) {
        if (!(l2 - l1 > tol * (l1 + l2) && steps < max_steps)) break;
        const double mid = 0.5 * (l1 + l2);
        if (vol[node] > vol_target) {
            l1 = mid;
            node = 2 * node + 1;
        } else {
            l2 = mid;
            node = 2 * node + 2;
        }
        lam = mid;
        vl = vol[(node - 1) / 2];
        steps++;
    }
    st[0] = l1;
    st[1] = l2;
    st[2] = lam;
    st[3] = vl;
    st[4] = (double)steps;
    st[5] = (l2 - l1 > tol * (l1 + l2) && steps < max_steps) ? 0.0 : 1.0;
}

// rho_new at the final multiplier, and block maxima of |rho_new - rho|
__global__ __launch_bounds__(256) void k_oc_apply(OcArgs A, const double *__restrict__ st, double *__restrict__ out,
                                                  double *__restrict__ part) {
    __shared__ double red[256];
    const double lam = st[2];
    double m = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < A.n; e += (int64_t)gridDim.x * 256) {
        const double r = A.rho[e];
        const double c = oc_new(r, A.dc[e], A.dv[e], lam, A.move, A.eta);
        out[e] = c;
        const double d = fabs(c - r);
        m = d > m || d != d ? d : m;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const double o = red[threadIdx.x + s];
            if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_oc_change(const double *__restrict__ part, int nblk, double *st) {
    __shared__ double red[256];
    double m = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) {
        const double o = part[b];
        if (o > m || o != o) m = o;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const double o = red[threadIdx.x + s];
            if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) st[6] = red[0];
}

}  // namespace

int oc_blocks(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (int)(b < kOcMaxBlocks ? (b > 0 ? b : 1) : kOcMaxBlocks);
}

hipError_t launch_oc_init(double *st, double lmax, hipStream_t s) {
    hipLaunchKernelGGL(k_oc_init, dim3(1), dim3(256), 0, s, st, lmax);
    return hipGetLastError();
}

hipError_t launch_oc_pass(const double *rho, const double *dc, const double *dv, int64_t n, double move, double eta,
                          double vol_target, double tol, int max_steps, double *st, double *part, hipStream_t s) {
    const int g = oc_blocks(n);
    const OcArgs A{rho, dc, dv, n, move, eta};
    hipLaunchKernelGGL(k_oc_eval, dim3(g), dim3(256), 0, s, A, st, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_oc_decide, dim3(1), dim3(1024), 0, s, part, g, vol_target, tol, max_steps, st);
    return hipGetLastError();
}

hipError_t launch_oc_apply(const double *rho, const double *dc, const double *dv, int64_t n, double move, double eta,
                           double *st, double *out, double *part, hipStream_t s) {
    const int g = oc_blocks(n);
    const OcArgs A{rho, dc, dv, n, move, eta};
    hipLaunchKernelGGL(k_oc_apply, dim3(g), dim3(256), 0, s, A, st, out, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_oc_change, dim3(1), dim3(256), 0, s, part, g, st);
    return hipGetLastError();
}

}  // namespace soptx
