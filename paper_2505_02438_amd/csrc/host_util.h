// Host-side helpers shared by the C ABI sources of libsoptx.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace soptx {

// Scratch of at least n doubles for work on (device, stream); `use` keeps
// independent buffers apart: 0 = reduction partials of the energy kernel,
// 1 = CG vectors, 2 = filter chain rule, 3 = OC bisection state and partials.  Work on one stream is ordered, so
// one buffer per (device, stream, use) is race-free.  Held until the process
// ends; grown (after a synchronisation of the stream) when a call needs more.
int get_workspace(int device, hipStream_t st, size_t n, double **out, int use);

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
