"""Algorithm 1 (Sec. 2.3): the optimality-criteria loop for minimum compliance
under a volume constraint, driven from the host; every numeric step runs in
the library's kernels (assembly with the Dirichlet rows, CG solve, element
sensitivities and compliance, filter, OC update).

Filters (Sec. 2.4): "sensitivity" filters dc; "density" assembles the filtered
density rho~ = F(rho) and takes dc and the volume sensitivity back through the
chain rule (so the constraint is the filtered volume, exactly, since F is
linear).  The loop stops when the largest density change of an update is at
most `tol` or after `max_iter` updates (the paper's runs use 0.01 and 200).
general: Q1 meshes whose elements are not affine, assembled and evaluated
with the Jacobian at every Gauss point.
Each CG solve starts from the previous iteration's displacement
(warm_start), stopping at ||r|| <= cg_rtol ||f||.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import api


@dataclasses.dataclass
class LoopResult:
    compliance: List[float]        # c = f^T u of the design entering each iteration
    volume_fraction: List[float]   # its (physical) volume fraction, from the previous update
    change: List[float]            # max |rho_new - rho| of each update
    cg_iterations: List[int]
    rho: "object"                  # final design variables (device tensor)


def run(mesh, mask, f, volfrac: float, rmin: float, filt: str = "sensitivity", rho0: Optional[float] = None,
        max_iter: int = 200, tol: float = 0.01, move: float = 0.2, eta: float = 0.5, cg_rtol: float = 1e-8,
        warm_start: bool = True, general: bool = False, material: Optional[api.Material] = None,
        stream=None) -> LoopResult:
    import torch
    if filt not in ("sensitivity", "density"):
        raise ValueError("filt is 'sensitivity' or 'density'")
    d = torch.device("cuda:0")
    pat = api.Pattern.from_mesh(mesh, general=general)
    flt = api.Filter.from_mesh(mesh, rmin)
    mat = material or api.Material(E0=1.0, Emin=1e-9, nu=0.3, p=3.0)
    n = mesh.n_cells
    # every tensor operation of the loop (allocations, u.zero_(), the reads of
    # c) is ordered on the loop's stream with the library's kernels
    with api._on(stream):
        vol = flt.volumes()                            # element measures (built on the host with H)
        v = torch.from_numpy(vol).to(d)
        total = float(vol.sum())
        mask_d = torch.from_numpy(np.asarray(mask, np.uint8)).to(d)
        f_d = torch.from_numpy(np.asarray(f, np.float64)).to(d)
        rho = torch.full((n,), volfrac if rho0 is None else rho0, dtype=torch.float64, device=d)
        dv = flt.density_backward(v, stream=stream) if filt == "density" else v
        K = torch.empty(pat.nnz, dtype=torch.float64, device=d)
        u = torch.zeros(pat.ndof, dtype=torch.float64, device=d)
        res = LoopResult([], [], [], [], None)
        vf = volfrac if rho0 is None else rho0      # a uniform design: the filter keeps it
        for _ in range(max_iter):
            phys = flt.density(rho, stream=stream) if filt == "density" else rho
            if general:
                pat.assemble_general(mat, phys, mask_d, out=K, stream=stream)
            else:
                pat.assemble(mat, phys, mask_d, out=K, stream=stream)
            if not warm_start:
                u.zero_()
            # the previous displacement starts the solve (the criterion is relative to ||f||)
            u, cg_it, _ = pat.pcg(K, f_d, u=u, rtol=cg_rtol, max_iter=50000, stream=stream)
            if general:
                dc, c = pat.evaluate_general(mat, phys, u, f=f_d, stream=stream)
            else:
                dc, c = pat.evaluate(mat, phys, u, f=f_d, stream=stream)
            if filt == "density":
                dcd = flt.density_backward(dc, stream=stream)
            else:
                dcd = flt.sensitivity(rho, dc, stream=stream)
            rho, info = api.oc_update(rho, dcd, dv, volfrac * total, move=move, eta=eta, stream=stream)
            res.compliance.append(float(c[1]))
            res.volume_fraction.append(vf)
            vf = info["volume"] / total                # sum dv rho_new: the next design's (filtered) volume
            res.change.append(info["change"])
            res.cg_iterations.append(cg_it)
            if info["change"] <= tol:
                break
        res.rho = rho
    return res

