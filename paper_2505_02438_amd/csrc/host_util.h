// Host-side helpers shared by the C ABI sources of libsoptx.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/soptx.h"

namespace soptx {

// Scratch of at least n doubles for work on (device, stream); `use` keeps
// independent buffers apart: 0 = reduction partials of the energy kernel,
// 1 = CG vectors, 2 = filter chain rule, 3 = OC bisection state and partials,
// 4 = element matrices of the per-quadrature-point assembly.  Work on one
// stream is ordered, so
// one buffer per (device, stream, use) is race-free.  Held until the process
// ends; when a call needs more, a larger buffer replaces it and the old one is
// kept (not freed), so that a HIP graph captured earlier on the stream, which
// holds the old address, still replays on valid memory.
int get_workspace(int device, hipStream_t st, size_t n, double **out, int use);

// Copy a host vector into a new device allocation recorded in `allocs` (freed
// with its handle); *dst = nullptr for an empty vector.  *bytes, if given,
// grows by the allocation's size.
template <class T>
int upload_vector(std::vector<void *> &allocs, const std::vector<T> &v, T **dst, hipStream_t st,
                  int64_t *bytes = nullptr) {
    *dst = nullptr;
    if (v.empty()) return SOPTX_OK;
    void *p = nullptr;
    if (hipMalloc(&p, v.size() * sizeof(T)) != hipSuccess) return SOPTX_E_OOM;
    allocs.push_back(p);
    if (hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st) != hipSuccess)
        return SOPTX_E_DEVICE;
    *dst = static_cast<T *>(p);
    if (bytes) *bytes += (int64_t)(v.size() * sizeof(T));
    return SOPTX_OK;
}

// Makes `dev` current for the lifetime of the guard and restores the
// previous device afterwards.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace soptx
