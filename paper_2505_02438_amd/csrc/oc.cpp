// C ABI of the OC update (arXiv 2505.02438, Sec. 2.3, Algorithm 1); the
// kernels are in oc.hip.  The host launches bisection passes (each advances
// up to kOcDepth steps on the device) in batches and reads the done flag
// after each batch.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/soptx_oc.h"
#include "host_util.h"
#include "internal.h"
#include "kernels.h"

using namespace soptx;

namespace {
constexpr int kPassesPerCheck = 4;
}

extern "C" int soptx_oc_update(int64_t n, const double *d_rho, const double *d_dc, const double *d_dv,
                               double vol_target, const soptx_oc_params *prm, double *d_rho_new,
                               soptx_oc_result *out, void *stream) {
    if (!prm || !out || n < 0 || !std::isfinite(vol_target)) return SOPTX_E_INVALID_ARG;
    if (!(prm->move > 0.0 && prm->move <= 1.0) || !(prm->eta > 0.0 && prm->eta <= 1.0) ||
        !(prm->lmax > 0.0 && std::isfinite(prm->lmax)) || !(prm->tol > 0.0 && prm->tol < 1.0) ||
        prm->max_steps < 1 || prm->max_steps > 1000)
        return SOPTX_E_INVALID_ARG;
    *out = soptx_oc_result{0.0, 0.0, 0.0, 0};
    if (n == 0) return SOPTX_OK;
    if (!d_rho || !d_dc || !d_dv || !d_rho_new || d_rho_new == d_rho || d_rho_new == d_dc || d_rho_new == d_dv)
        return SOPTX_E_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SOPTX_E_DEVICE;
    double *ws = nullptr;
    int rc = get_workspace(dev, st, (size_t)kOcNodes * kOcMaxBlocks + 8, &ws, 3);
    if (rc) return rc;
    double *state = ws, *part = ws + 8;
    if (launch_oc_init(state, prm->lmax, st) != hipSuccess) return SOPTX_E_DEVICE;
    const int max_passes = (prm->max_steps + kOcDepth - 1) / kOcDepth;
    double h[8];
    for (int p = 0; p < max_passes;) {
        for (int q = 0; q < kPassesPerCheck && p < max_passes; q++, p++)
            if (launch_oc_pass(d_rho, d_dc, d_dv, n, prm->move, prm->eta, vol_target, prm->tol, prm->max_steps,
                               state, part, st) != hipSuccess)
                return SOPTX_E_DEVICE;
        if (hipMemcpyAsync(h, state, 7 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return SOPTX_E_DEVICE;
        if (h[5] != 0.0) break;
    }
    if (launch_oc_apply(d_rho, d_dc, d_dv, n, prm->move, prm->eta, state, d_rho_new, part, st) != hipSuccess)
        return SOPTX_E_DEVICE;
    if (hipMemcpyAsync(h, state, 7 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return SOPTX_E_DEVICE;
    out->lambda = h[2];
    out->volume = h[3];
    out->steps = (int32_t)h[4];
    out->change = h[6];
    return SOPTX_OK;
}
