// Fixed-order block reduction shared by the kernels that produce block
// partial sums (compliance, CG dot products).
#pragma once
#include <hip/hip_runtime.h>

namespace soptx {

// Sum over a block of 256 threads in a fixed order (tree); the result is
// returned to every thread.  red: 256 doubles of LDS.
static __device__ __forceinline__ double block_sum_256(double x, double *red) {
    __syncthreads();  // red may still be read by a previous call
    red[threadIdx.x] = x;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    return red[0];
}

}  // namespace soptx
