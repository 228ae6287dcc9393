"""Helpers for GPU parity tests: device copies and the error metrics.

Error metrics (the reading of "rel. err" used throughout):
* K: row-scaled  max_r max_{k in r} |dK_k| / max_{k in r} |Kref_k|
  (entries may cancel to ~0 structurally; rows differ by the 1e9 contrast).
* dc: condition-scaled |d dc_e| / (|E'_e| |u_e|^T |K_e^0| |u_e|), the forward
  error scale of the quadratic form; the plain relative error is reported too.
* c: |dc| / sum_e E_e |u_e|^T |K_e^0| |u_e|.
"""
import numpy as np
import torch

from oracle import oracle as O


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def host(t):
    return t.detach().to("cpu").numpy()


def row_scaled_err(rp, Kx, Kref):
    rp = np.asarray(rp, dtype=np.int64)
    n = rp.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    den = np.zeros(n)
    np.maximum.at(den, rows, np.abs(Kref))
    num = np.zeros(n)
    np.maximum.at(num, rows, np.abs(Kx - Kref))
    ok = den > 0
    return float(np.max(num[ok] / den[ok])) if ok.any() else 0.0


def abs_energy(mesh, u, idx):
    """|u_e|^T |K_e^0| |u_e| for the elements idx (oracle element matrices)."""
    d, nen = mesh.dim, mesh.nen
    out = np.zeros(len(idx))
    for k, e in enumerate(idx):
        Ke = O.element_ke0(mesh.elem, mesh.coords[mesh.cells[e]], 0.3)
        dofs = (d * mesh.cells[e][:, None] + np.arange(d)).ravel()
        ue = np.abs(u[dofs])
        out[k] = ue @ np.abs(Ke) @ ue
    return out


def dE(rho, p=3.0, E0=1.0, Emin=1e-9):
    return p * rho ** (p - 1) * (E0 - Emin)


def E(rho, p=3.0, E0=1.0, Emin=1e-9):
    return Emin + rho ** p * (E0 - Emin)
