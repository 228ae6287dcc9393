"""Plain FP64 CPU oracle of the optimality-criteria (OC) update (Sec. 2.3,
the update factor B_e, the clamped heuristic update and Algorithm 1's
bisection on the multiplier lambda).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product path never does.
It imports nothing from the HIP package.

Definitions followed:
* B_e(lambda) = -dc_e / (lambda dv_e), dc the objective's and dv the volume
  constraint's sensitivities with respect to the design variables; a
  positive dc_e (not produced by compliance, whose sensitivities are <= 0)
  is read as B_e = 0;
* rho_new_e = rho_e B_e^eta clamped to [max(0, rho_e - m), min(1, rho_e + m)],
  the three cases of the update with move limit m and damping eta;
* vol(lambda) = sum_e dv_e rho_new_e(lambda), non-increasing in lambda;
* bisection: l1 = 0, l2 = lmax; while l2 - l1 > tol (l1 + l2) (and fewer than
  max_steps steps): mid = (l1 + l2) / 2, rho_new at lambda = mid, and l1 = mid
  if vol(mid) > V* else l2 = mid.  The result is rho_new at the last mid.
* change = max_e |rho_new_e - rho_e| (the stopping test of Algorithm 1).
"""
from __future__ import annotations

import math

import numpy as np


def oc_candidate(rho, dc, dv, lam: float, move: float, eta: float) -> np.ndarray:
    """rho_new(lambda) for every element."""
    rho = np.asarray(rho, np.float64)
    dc = np.asarray(dc, np.float64)
    dv = np.asarray(dv, np.float64)
    B = np.maximum(0.0, -dc) / (lam * dv)
    if eta == 0.5:
        Be = np.sqrt(B)
    elif eta == 1.0:
        Be = B
    else:
        Be = B ** eta
    cand = rho * Be
    lo = np.maximum(0.0, rho - move)
    hi = np.minimum(1.0, rho + move)
    return np.minimum(hi, np.maximum(lo, cand))


def volume(dv, rho_new) -> float:
    """sum_e dv_e rho_new_e, correctly rounded (math.fsum of the rounded products)."""
    return math.fsum((np.asarray(dv, np.float64) * np.asarray(rho_new, np.float64)).tolist())


def oc_update(rho, dc, dv, vol_target: float, move: float = 0.2, eta: float = 0.5, lmax: float = 1e9,
              tol: float = 1e-3, max_steps: int = 200):
    """Returns (rho_new, lambda, vol(lambda), steps, change)."""
    l1, l2 = 0.0, float(lmax)
    steps = 0
    lam, rn, vol = None, None, None
    while l2 - l1 > tol * (l1 + l2) and steps < max_steps:
        mid = 0.5 * (l1 + l2)
        rn = oc_candidate(rho, dc, dv, mid, move, eta)
        vol = volume(dv, rn)
        if vol > vol_target:
            l1 = mid
        else:
            l2 = mid
        lam = mid
        steps += 1
    change = float(np.max(np.abs(rn - np.asarray(rho, np.float64)))) if len(rn) else 0.0
    return rn, lam, vol, steps, change
