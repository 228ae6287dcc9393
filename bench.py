#!/usr/bin/env python
"""Throughput of SIMP assembly + sensitivity + compliance on one MI355X.

Workload: the 3D cantilever of 120 x 40 x 40 unit Q1 hexahedra (192,000
elements, 610,203 dofs, 47,568,609 stored K entries), rho ~ Beta(2, 2), p = 3,
E0 = 1, Emin = 1e-9, nu = 0.3, x = 0 face clamped, synthetic u ~ N(0, 1)
(zero on fixed dofs).  One step = soptx_step (FP64 CSR values with the
clamped face's rows and columns, from a Dirichlet table bound once) +
soptx_evaluate (dc and c), all inputs resident in HBM, three rotating output
buffers so that writes do not hit in the 256 MB MALL.  HIP events on the
bench stream time the assembly (its roofline) and the evaluation of every
step.  A second timed region replays the same step as a captured HIP graph
(graph_value, graph_ms_per_step).  Then: the FP32 form of the same step, the
labelled rows (the same cantilever sheared, so every J^-1 is full; P1
triangles 600x200; P2 tetrahedra 48^3 in both forms), the solve, filter, OC
and loop measurements, serving, and the CPU oracle on a bounded sample.
Prints one JSON line.

    python bench.py [--gpus 1] [--steps 50] [--warmup 5]

--workload runs the headline step on one of the other configurations (P1
triangles 600x200, P2 tetrahedra 48^3, Q1 hexahedra 96^3) instead.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E datasheet peak
METRIC = "elements assembled+sensitized/sec, % HBM roofline; p50/p99 request latency"
COUNTERS = os.path.join(ROOT, "profiles", "k_assemble_hex8_120x40x40_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2505_02438_amd", "csrc", "kernels.hip")


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


# --workload: the default is the configuration the metric is quoted on; the
# others are the parity-test configurations, measured the same way
WORKLOADS = {
    "hex120x40x40": ("3D cantilever 120x40x40 unit Q1 hexahedra (192,000 elements, 610,203 dofs, "
                     "47,568,609 K entries), rho~Beta(2,2), p=3, nu=0.3, x=0 face clamped, u~N(0,1)",
                     lambda I: I.cantilever_hex()),
    "tri600x200": ("2D cantilever 600x200 squares x 2 jittered P1 triangles (240,000 elements, 241,602 dofs, "
                   "3,369,604 K entries), rho~U(0.001,1), p=3, nu=0.3, plane stress, x=0 edge clamped, u~N(0,1)",
                   lambda I: I.cantilever_tri()),
    "p2box48": ("3D box 48^3 cubes x 6 jittered Kuhn P2 tetrahedra (663,552 elements, 2,738,019 dofs, "
                "231,797,385 K entries), rho~U(0.001,1), p=3, nu=0.3, x=0 face clamped, u~N(0,1)",
                lambda I: I.box_p2()),
    "hex120x40x40_sheared": ("the 120x40x40 cantilever mapped by x -> A x, A = [[1, .3, .1], [-.2, 1, .25], "
                             "[.15, -.1, 1]]: every element affine with a full J^-1 (the general affine "
                             "contraction), rho, u and supports as the headline", lambda I: I.cantilever_hex(skew="global")),
    "hex120x40x40_renumbered": ("the headline cantilever with its nodes and elements renumbered by a seeded "
                                "permutation (seed 17): the plan takes its canonical order",
                                lambda I: I.renumber(I.cantilever_hex(), 17)),
    "hex96": ("3D cube 96^3 unit Q1 hexahedra (884,736 elements, 2,738,019 dofs, 217,238,121 K entries; the "
              "largest serving request), rho~Beta(2,2), p=3, nu=0.3, x=0 face clamped, u~N(0,1)",
              lambda I: I.cantilever_hex(96, 96, 96)),
}
STEP = "; step = assemble (FP64 CSR) with the Dirichlet rows/columns + sensitivity + compliance"


def algorithmic_bytes(n_nodes, n_cells, nnz, dim, nen, ndof):
    """Minimum bytes each call must move (FP64 form).

    assemble with Dirichlet: write K values (nnz*8); read rho (NC*8),
    coordinates (n_nodes*dim*8), cells (NC*nen*4) and the fixed-dof mask
    (ndof bytes).
    evaluate: read rho, u (ndof*8), coordinates, cells; write dc (NC*8).
    """
    asm = nnz * 8 + n_cells * 8 + n_nodes * dim * 8 + n_cells * nen * 4 + ndof
    ev = n_cells * 8 + ndof * 8 + n_nodes * dim * 8 + n_cells * nen * 4 + n_cells * 8
    return asm, ev


def solve_run(pat, m, K, f, stream, rtol, reps=20):
    """The equilibrium solve on the assembled K (Dirichlet applied): the SpMV
    timed with HIP events on the bench stream against its algorithmic bytes
    (K values, one neighbour id per DIM x DIM block, row offsets, x read, y
    written), and one full preconditioned CG solve."""
    import torch
    x = torch.ones(pat.ndof, dtype=torch.float64, device=K.device)
    y = torch.empty_like(x)
    ms = []
    for _ in range(reps + 3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        pat.spmv(K, x, out=y, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    spmv_s = statistics.mean(ms[3:]) / 1e3
    nbytes = pat.nnz * 8 + (pat.nnz // (m.dim * m.dim)) * 4 + m.n_nodes * 2 * 4 + 2 * pat.ndof * 8
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, iters, rel = pat.pcg(K, f, rtol=rtol, max_iter=50000, stream=stream)
    torch.cuda.synchronize()
    solve_s = time.perf_counter() - t0
    return {"spmv_avg_ms": spmv_s * 1e3, "spmv_algorithmic_bytes": nbytes,
            "spmv_achieved_GBs": nbytes / spmv_s / 1e9, "spmv_frac_of_hbm_peak": nbytes / spmv_s / 1e9 / HBM_PEAK_GBS,
            "pcg_rtol": rtol, "pcg_iterations": iters, "pcg_relres": rel, "pcg_seconds": solve_s,
            "pcg_ms_per_iteration": solve_s / max(iters, 1) * 1e3}


FILTER_RADIUS = {2: 6.0, 3: 1.5}   # the radii of the paper's 2D and 3D examples


def filter_run(pat, m, mat, rho, K, stream, beta=8.0, reps=20):
    """The filter step on the workload's mesh at the paper's radius: the
    density filter with the Heaviside projection, the sensitivity filter and
    the chain rule, each timed with HIP events on the bench stream.  An
    assembly runs between two filter calls, as in an optimisation step, so
    H is not left in the last-level cache by the previous call."""
    import torch
    from paper_2505_02438_amd import api
    rmin = FILTER_RADIUS[m.dim]
    t0 = time.perf_counter()
    flt = api.Filter.from_mesh(m, rmin)
    build_s = time.perf_counter() - t0
    n = flt.n
    rt = torch.empty(n, dtype=torch.float64, device=rho.device)
    rb, dc, dco, gr = (torch.empty_like(rt) for _ in range(4))
    dc.fill_(-1.0)
    torch.cuda.synchronize()
    names = ("density_heaviside", "sensitivity", "chain_rule")
    ms = {k: [] for k in names}
    for r in range(reps + 3):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        ev[0].record(stream)
        flt.density(rho, beta=beta, rho_tilde=rt, rho_bar=rb, stream=stream)
        ev[1].record(stream)
        pat.assemble(mat, rho, None, out=K, stream=stream)
        ev[2].record(stream)
        flt.sensitivity(rho, dc, out=dco, stream=stream)
        ev[3].record(stream)
        pat.assemble(mat, rho, None, out=K, stream=stream)
        ev[4].record(stream)
        flt.density_backward(dc, rho_tilde=rt, beta=beta, out=gr, stream=stream)
        ev[5].record(stream)
        torch.cuda.synchronize()
        if r >= 3:
            for k, (a, b) in zip(names, ((0, 1), (2, 3), (4, 5))):
                ms[k].append(ev[a].elapsed_time(ev[b]))
    # algorithmic bytes: each distinct vector read or written once, plus H
    # once (int32 column + FP64 weight per entry, row offsets) in the CSR form;
    # the stencil form reads no H (its table of offsets is a few hundred bytes)
    hbytes = 0 if flt.stencil_size else flt.nnz * 12 + (n + 1) * 4
    vec = {"density_heaviside": 5, "sensitivity": 4, "chain_rule": 7}
    out = {"rmin": rmin, "beta": beta, "elements": n, "nnz": flt.nnz,
           "form": f"stencil ({flt.stencil_size} offsets)" if flt.stencil_size else "csr",
           "rows_per_block": flt.rows_per_block, "build_s": build_s}
    for k in names:
        avg = statistics.mean(ms[k]) / 1e3
        nb = hbytes + vec[k] * n * 8
        out[k] = {"avg_ms": avg * 1e3, "algorithmic_bytes": nb, "achieved_GBs": nb / avg / 1e9,
                  "frac_of_hbm_peak": nb / avg / 1e9 / HBM_PEAK_GBS}
    return out


def oc_run(pat, n, dc, stream, reps=20):
    """The OC update alone on the workload's elements: densities and
    sensitivities of the bench step, unit constraint sensitivities, volume
    fraction 0.3 (the 3D cantilever's), m = 0.2, eta = 0.5, bisection to a
    relative bracket of 1e-3 from [0, 1e9].  Host-synchronous calls, wall time."""
    import torch
    from paper_2505_02438_amd import api
    rho = torch.full((n,), 0.3, dtype=torch.float64, device=dc.device)
    ones = torch.ones_like(rho)
    out = torch.empty_like(rho)
    torch.cuda.synchronize()
    ts, info = [], None
    for r in range(reps + 3):
        t0 = time.perf_counter()
        _, info = api.oc_update(rho, dc, ones, 0.3 * n, out=out, stream=stream)
        ts.append(time.perf_counter() - t0)
    return {"avg_ms": statistics.mean(ts[3:]) * 1e3, "bisection_steps": info["steps"],
            "device_passes": (info["steps"] + 3) // 4, "lambda": info["lambda"]}


def to_loop_run(iters, stream, rtol=1e-8):
    """Whole optimisation iterations (Algorithm 1) on the GPU, on the 3D
    cantilever of the paper's CPU/GPU comparison: 120 x 40 x 8 unit Q1
    hexahedra, x = 0 face clamped, f_y = -1 at the nodes of the edge x = 120,
    y = 0; volume fraction 0.3 from a uniform 0.3; sensitivity filter r = 3.0;
    OC with m = 0.2, eta = 0.5; CG from the previous iteration's displacement
    to ||r|| <= rtol ||f||.  An iteration: assemble K with the Dirichlet rows, solve, element
    sensitivities and compliance, sensitivity filter, OC update."""
    import torch
    from paper_2505_02438_amd import api
    from paper_2505_02438_amd import inputs as I
    mesh = I.hex_grid(120, 40, 8)
    mask_h, f_h = I.clamp_x0_bc(mesh)
    d = torch.device("cuda:0")
    pat = api.Pattern.from_mesh(mesh)
    flt = api.Filter.from_mesh(mesh, 3.0)
    mat = api.Material(E0=1.0, Emin=1e-9, nu=0.3, p=3.0)
    n = mesh.n_cells
    mask = torch.from_numpy(mask_h).to(d)
    f = torch.from_numpy(f_h).to(d)
    rho = torch.full((n,), 0.3, dtype=torch.float64, device=d)
    ones = torch.ones_like(rho)
    K = torch.empty(pat.nnz, dtype=torch.float64, device=d)
    u = torch.zeros(pat.ndof, dtype=torch.float64, device=d)
    torch.cuda.synchronize()
    times, cgs, cs = [], [], []
    t_all = time.perf_counter()
    for it in range(iters):
        t0 = time.perf_counter()
        pat.assemble(mat, rho, mask, out=K, stream=stream)
        u, cg_it, _ = pat.pcg(K, f, u=u, rtol=rtol, max_iter=50000, stream=stream)   # from the last u
        dc, c = pat.evaluate(mat, rho, u, f=f, stream=stream)
        dcf = flt.sensitivity(rho, dc, stream=stream)
        rho, info = api.oc_update(rho, dcf, ones, 0.3 * n, move=0.2, eta=0.5, stream=stream)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        cgs.append(cg_it)
        cs.append(float(c[1]))
    total = time.perf_counter() - t_all
    return {"mesh": "120x40x8 Q1 hex", "elements": n, "ndof": pat.ndof, "iterations": iters, "total_s": total,
            "first_iter_s": times[0], "avg_iter_s": (total - times[0]) / max(iters - 1, 1),
            "cg_rtol": rtol, "cg_iterations_avg": statistics.mean(cgs), "cg_iterations_last": cgs[-1],
            "compliance_first": cs[0], "compliance_last": cs[-1],
            "volume_fraction_last": float(rho.sum()) / n}


def general_run(stream, reps=20, two_d=False):
    """Assembly with per-quadrature-point geometry on general Q1 cells: the 3D
    cantilever's 120 x 40 x 40 hexahedra with every interior node moved by
    U(-0.2, 0.2) per coordinate (seed 54), rho and u of the main workload; or
    (two_d) the 2D cantilever's 600 x 200 quadrilaterals jittered the same
    way (seed 57), rho ~ U(0.001, 1), clamped left edge.  FP64, Dirichlet
    rows; HIP events on the bench stream."""
    import ctypes
    import numpy as np
    import torch
    from paper_2505_02438_amd import _lib, api
    from paper_2505_02438_amd import inputs as I
    if two_d:
        rng = np.random.default_rng(57)
        m = I.jitter_interior(I.quad_grid(600, 200), 0.2, rng)
        rho_h = rng.uniform(0.001, 1.0, m.n_cells)
        mask_h, _ = I.cantilever2d_bc(m, load="mid_right")
        u_h = I.synthetic_u(rng, mask_h)
        mat = api.Material()
        mesh_desc = "600x200 quadrilaterals, interior nodes jittered by 0.2"
    else:
        pr = I.cantilever_hex()
        m = I.jitter_interior(pr.mesh, 0.2, np.random.default_rng(54))
        rho_h, mask_h, u_h = pr.rho, pr.mask, pr.u
        mat = api.Material(E0=pr.E0, Emin=pr.Emin, nu=pr.nu, p=pr.p)
        mesh_desc = "120x40x40 hexahedra, interior nodes jittered by 0.2"
    t0 = time.perf_counter()
    pat = api.Pattern.from_mesh(m, general=True)
    build_s = time.perf_counter() - t0
    rho = torch.from_numpy(rho_h).cuda()
    mask = torch.from_numpy(mask_h).cuda()
    K = torch.empty(pat.nnz, dtype=torch.float64, device="cuda")
    L = _lib.lib()
    in_lds = ctypes.c_int32(-1)

    def time_assembly(variant):
        _lib.check(L.soptx_debug_set_general_variant(variant), "general variant")
        try:
            _lib.check(L.soptx_debug_general_path(pat._h, ctypes.byref(in_lds)), "general path")
            torch.cuda.synchronize()
            ms = []
            for r in range(reps + 3):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                pat.assemble_general(mat, rho, mask, out=K, stream=stream)
                b.record(stream)
                torch.cuda.synchronize()
                ms.append(a.elapsed_time(b))
        finally:
            L.soptx_debug_set_general_variant(-1)
        return statistics.mean(ms[3:]) / 1e3, in_lds.value
    avg_ke, _ = time_assembly(0)
    avg_stage, _ = time_assembly(1)
    avg, form = time_assembly(-1)
    # the default form back to back: the fastest of three bursts of `reps`
    # calls between one pair of events (as the headline's roofline kernel time)
    bursts = []
    for rep in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for r in range(reps):
            pat.assemble_general(mat, rho, mask, out=K, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        bursts.append(a.elapsed_time(b) / reps / 1e3)
    avg_b2b = min(bursts)
    u = torch.from_numpy(u_h).cuda()
    dc = torch.empty(m.n_cells, dtype=torch.float64, device="cuda")
    c = torch.zeros(2, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    ev = []
    for r in range(reps + 3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        pat.evaluate_general(mat, rho, u, dc=dc, c=c, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        ev.append(a.elapsed_time(b))
    ev_avg = statistics.mean(ev[3:]) / 1e3
    kbytes = pat.nnz * 8
    return {"mesh": mesh_desc, "elements": m.n_cells,
            "form": {1: "in LDS on the plan's node groups, sums in registers (k_assemble_point)",
                     2: "in LDS on the plan's node groups, sums in an LDS stage (k_assemble_quad)"}.get(
                         form, "element matrices through memory (k_ke_general, k_gather_general)"),
            "avg_ms": avg * 1e3, "avg_ms_back_to_back": avg_b2b * 1e3,
            "avg_ms_how": "avg_ms: HIP events around each call; avg_ms_back_to_back: the fastest of three "
                          "bursts of %d calls between one pair of events" % reps,
            "elements_per_s": m.n_cells / avg, "K_bytes": kbytes,
            "K_write_GBs": kbytes / avg / 1e9, "stage_form_avg_ms": avg_stage * 1e3,
            "element_matrix_form_avg_ms": avg_ke * 1e3,
            "evaluate_avg_ms": ev_avg * 1e3,
            "step_elements_per_s": m.n_cells / (avg + ev_avg), "pattern_build_s": build_s}


def hex27_run(stream, reps=10):
    """Q2 hexahedra (27 nodes, 3 x 3 x 3 Gauss points) with per-point geometry:
    the curved 60 x 20 x 20 cantilever (cubes of side 2 over the 120 x 40 x 40
    box, the Q1 cantilever's node lattice; interior nodes jittered by 0.15,
    seed 1005), rho ~ Beta(2, 2), FP64, Dirichlet rows; HIP events on the
    bench stream.  Byte model of the assembly: element matrices written and
    read back (n_cells 27^2 9 doubles each way), K written, the contribution
    table (gptr, gent, gnode) read."""
    import torch
    from paper_2505_02438_amd import api
    from paper_2505_02438_amd import inputs as I
    pr = I.cantilever_hex27()
    m = pr.mesh
    t0 = time.perf_counter()
    pat = api.Pattern.from_mesh(m, general=True)
    build_s = time.perf_counter() - t0
    mat = api.Material(E0=pr.E0, Emin=pr.Emin, nu=pr.nu, p=pr.p)
    rho = torch.from_numpy(pr.rho).cuda()
    mask = torch.from_numpy(pr.mask).cuda()
    K = torch.empty(pat.nnz, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    def timed(fn):
        ms = []
        for r in range(reps + 3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        return statistics.mean(ms[3:]) / 1e3

    avg = timed(lambda: pat.assemble_general(mat, rho, mask, out=K, stream=stream))
    u = torch.from_numpy(pr.u).cuda()
    dc = torch.empty(m.n_cells, dtype=torch.float64, device="cuda")
    c = torch.zeros(2, dtype=torch.float64, device="cuda")
    ev_avg = timed(lambda: pat.evaluate_general(mat, rho, u, dc=dc, c=c, stream=stream))
    ke_bytes = m.n_cells * 27 * 27 * 9 * 8
    nblk = pat.nnz // 9
    table_bytes = 4 * (nblk + 1) + 4 * m.n_cells * 27 * 27 + 4 * nblk
    moved = 2 * ke_bytes + pat.nnz * 8 + table_bytes
    return {"mesh": "60x20x20 Q2 hexahedra (side 2), interior nodes jittered by 0.15", "elements": m.n_cells,
            "ndof": pat.ndof, "nnz": pat.nnz, "avg_ms": avg * 1e3, "elements_per_s": m.n_cells / avg,
            "bytes_moved": moved, "effective_GBs": moved / avg / 1e9, "evaluate_avg_ms": ev_avg * 1e3,
            "step_elements_per_s": m.n_cells / (avg + ev_avg), "pattern_build_s": build_s}


def paper_runs():
    """Whole optimisation runs (Algorithm 1) of the paper's examples, on the
    GPU: final compliance and volume fraction, iterations and wall time, with
    the values the paper prints beside them (tests/golden/paper_values.json)."""
    from paper_2505_02438_amd import inputs as I
    from paper_2505_02438_amd import loop
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_values.json")))
    cases = [
        ("cantilever2d_160x100_rho0.4", lambda: I.quad_grid(160, 100), lambda m: I.cantilever2d_bc(m), 0.4, 6.0,
         "sensitivity", 0.4, golden["loop_cantilever2d_160x100_rho0.4"]["printed"][-1][1:]),
        ("cantilever2d_160x100_rho1", lambda: I.quad_grid(160, 100), lambda m: I.cantilever2d_bc(m), 0.4, 6.0,
         "sensitivity", 1.0, golden["loop_cantilever2d_160x100_rho1"]["printed"][-1][1:]),
        ("mbb_150x50_quad", lambda: I.quad_grid(150, 50), I.mbb_bc, 0.5, 6.0, "sensitivity", None,
         golden["loop_mbb_150x50_quad"]["final"]),
        ("mbb_150x50_tri", lambda: I.tri_grid(150, 50), I.mbb_bc, 0.5, 6.0, "sensitivity", None,
         golden["loop_mbb_150x50_tri"]["final"]),
        ("cantilever3d_60x20x4", lambda: I.hex_grid(60, 20, 4), I.clamp_x0_bc, 0.3, 1.5, "sensitivity", None,
         golden["loop_cantilever3d_60x20x4"]["printed"][-1][1:]),
        ("mbb_150x50_density_filter", lambda: I.quad_grid(150, 50), I.mbb_bc, 0.5, 6.0, "density", None,
         golden["loop_mbb_150x50_density_filter"]["final_density_filter"]),
    ]
    out = []
    for name, mk, bc, vf, r, filt, rho0, printed in cases:
        m = mk()
        mask, f = bc(m)
        t0 = time.perf_counter()
        res = loop.run(m, mask, f, vf, r, filt=filt, rho0=rho0)
        out.append({"case": name, "filter": f"{filt} r={r}", "iterations": len(res.compliance),
                    "seconds": time.perf_counter() - t0, "compliance": round(res.compliance[-1], 4),
                    "volume_fraction": round(res.volume_fraction[-1], 4), "paper": printed})
    return out


def serving_run(count, slots=4, budget=32 << 30):
    """Serving form: seeded requests (2D Q1 n^2, n in 32..512; 3D Q1 n^3,
    n in 16..96; p in {3, 4}), first as a burst (saturated elements/s), then
    with Poisson arrivals at 0.7 x that rate (p50/p99 latency).  Inputs are
    resident in HBM when the run starts, as in the plain step; the burst is
    also run with every request's inputs copied from pinned host memory at
    launch (PCIe included)."""
    from paper_2505_02438_amd import serving as S

    def run(reqs, pcie=False):
        ex = S.GpuExecutor(slots, pcie=pcie)
        ex.prepare(reqs)
        ex.t0 = time.perf_counter()
        return S.latency_stats(S.Scheduler(ex, slots, budget).run(reqs))

    st_b = run(S.make_requests(count))
    lam = 0.7 * st_b["elements_per_s"]
    st_p = run(S.make_requests(count, rate_elems_per_s=lam))
    st_x = run(S.make_requests(count), pcie=True)
    return {"requests": count, "slots": slots, "hbm_budget_bytes": budget,
            "burst_elements_per_s": st_b["elements_per_s"], "burst_makespan_s": st_b["makespan_s"],
            "poisson_lambda_elements_per_s": lam, "p50_ms": st_p["p50_ms"], "p99_ms": st_p["p99_ms"],
            "poisson_elements_per_s": st_p["elements_per_s"],
            "burst_pcie_elements_per_s": st_x["elements_per_s"], "burst_pcie_makespan_s": st_x["makespan_s"]}


class StepState:
    """Device inputs of one workload, its Dirichlet table bound once, and
    `nbuf` rotating outputs (so that successive steps do not write K into
    lines the 256 MB MALL still holds)."""

    def __init__(self, pr, pat, prec, stream, nbuf=3):
        import torch
        from paper_2505_02438_amd import api
        dev = torch.device("cuda:0")
        self.pat, self.prec, self.nbuf = pat, prec, nbuf
        self.mat = api.Material(E0=pr.E0, Emin=pr.Emin, nu=pr.nu, p=pr.p)
        rdt = torch.float64 if prec == api.FP64 else torch.float32
        with torch.cuda.stream(stream):
            self.rho = torch.from_numpy(pr.rho).to(dev).to(rdt)
            self.u = torch.from_numpy(pr.u).to(dev)
            self.Ks = [torch.empty(pat.nnz, dtype=torch.float64, device=dev) for _ in range(nbuf)]
            self.dcs = [torch.empty(pat.n_cells, dtype=rdt, device=dev) for _ in range(nbuf)]
            self.cs = [torch.zeros(2, dtype=torch.float64, device=dev) for _ in range(nbuf)]
        self.bc = api.Dirichlet(pat, pr.mask, stream=stream)
        torch.cuda.synchronize()

    def fused(self, i, stream):
        """One step in one call: soptx_step with u, dc and c (the energies,
        then K with the Dirichlet rows and columns; the assembly kernel adds
        the partials of c)."""
        b = i % self.nbuf
        self.pat.step(self.mat, self.rho, self.u, bc=self.bc, K=self.Ks[b], dc=self.dcs[b], c=self.cs[b],
                      prec=self.prec, stream=stream)

    def assemble_only(self, i, stream):
        """K with the Dirichlet rows and columns alone (soptx_step without u)."""
        b = i % self.nbuf
        self.pat.step(self.mat, self.rho, bc=self.bc, K=self.Ks[b], prec=self.prec, stream=stream)

    def step(self, i, stream, ev=None):
        """The same step as two calls, for the stage times: K with the
        Dirichlet rows and columns (soptx_step, the bound table), then dc and c
        (soptx_evaluate); events around each."""
        b = i % self.nbuf
        if ev is not None:
            ev[0].record(stream)
        self.pat.step(self.mat, self.rho, bc=self.bc, K=self.Ks[b], prec=self.prec, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        self.pat.evaluate(self.mat, self.rho, self.u, dc=self.dcs[b], c=self.cs[b], prec=self.prec, stream=stream)
        if ev is not None:
            ev[2].record(stream)


def spin_up(st, stream, seconds):
    """Untimed steps for `seconds` of wall time, so that the timed steps run at
    the clocks a busy GPU holds (after the seconds of host-only work of the
    pattern build the GPU idles at lower clocks, and a few warm-up steps of
    0.1 ms do not bring them back)."""
    import torch
    t0 = time.perf_counter()
    i = 0
    while time.perf_counter() - t0 < seconds:
        for _ in range(20):
            st.fused(i, stream)
            i += 1
        torch.cuda.synchronize()
    return i


def pct(xs):
    xs = sorted(xs)
    n = len(xs)
    return {"p10": xs[n // 10], "p50": xs[n // 2], "p90": xs[min(n - 1, (9 * n) // 10)]}


def timed_steps(st, stream, steps, warmup):
    """warmup untimed steps, then `steps` fused steps (one call each, no
    events between them) timed by the wall clock, synchronised on both sides.
    Then the stage-split region: `steps` more steps as two calls with HIP
    events on the bench stream around the assembly and the evaluation of each
    (timing events between kernels cost several microseconds per step, so the
    timed region has none)."""
    import torch
    for i in range(warmup):
        st.fused(i, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        st.fused(i, stream)
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t0
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for i in range(steps):
        st.step(i, stream, events[i])
    torch.cuda.synchronize()
    asm_ms = [e[0].elapsed_time(e[1]) for e in events]
    ev_ms = [e[1].elapsed_time(e[2]) for e in events]
    # the assembly alone, `steps` launches back to back between one pair of
    # events: its average launch duration without a timing event next to each.
    # The fastest of three such bursts: a pause of the host while it enqueues
    # can leave the GPU idle inside a burst's window and only lengthens it
    bursts = []
    for rep in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for i in range(steps):
            st.assemble_only(i, stream)
        b.record(stream)
        torch.cuda.synchronize()
        bursts.append(a.elapsed_time(b) / steps)
    st.asm_burst_ms = min(bursts)
    # Each of the two is an upper bound on the kernel's duration: the events
    # around each call hold the dispatch gap before the kernel, and back to
    # back a launch's workgroups start as the previous launch's finish CU by
    # CU, out of the groups' lockstep order (on a warm box 89 vs 82 us).
    # The kernel time is the smaller
    st.asm_each_ms = statistics.median(asm_ms)
    st.asm_kernel_ms = min(st.asm_burst_ms, st.asm_each_ms)
    return total_s, asm_ms, ev_ms


def row_scaled_err(rows, K, Kref):
    """max over stored entries of |K - Kref| / max |Kref| of the entry's row (on the GPU)."""
    import torch
    rmax = torch.zeros(int(rows.max()) + 1, dtype=torch.float64, device=K.device)
    rmax.scatter_reduce_(0, rows, Kref.abs(), "amax")
    return float(((K - Kref).abs() / rmax[rows].clamp_min(1e-300)).max())


def labelled_run(name, desc, pr, stream, steps, warmup, precs, extra=None):
    """The headline step (assembly with Dirichlet, then dc and c) on another
    mesh: HIP events per stage, the assembly kernel against its algorithmic
    bytes, in each precision form of precs (FP32 also gives its error against
    the FP64 result of the same inputs)."""
    import torch
    from paper_2505_02438_amd import api
    m = pr.mesh
    t0 = time.perf_counter()
    pat = api.Pattern.from_mesh(m)
    build_s = time.perf_counter() - t0
    stats = pat.stats()
    asm_bytes, ev_bytes = algorithmic_bytes(m.n_nodes, m.n_cells, pat.nnz, m.dim, m.nen, m.ndof)
    out = {"workload": desc, "elements": m.n_cells, "ndof": pat.ndof, "nnz": pat.nnz,
           "pattern_build_s": build_s, "groups": stats["n_groups"], "signatures": stats["n_signatures"],
           "groups_with_rank_table": stats["n_groups_ranked"]}
    if extra:
        out.update(extra)
    states = {}
    for prec in precs:
        st = states[prec] = StepState(pr, pat, prec, stream)
        spin_up(st, stream, 0.2)
        total_s, asm_ms, ev_ms = timed_steps(st, stream, steps, warmup)
        a = st.asm_kernel_ms / 1e3
        key = "fp64" if prec == api.FP64 else "fp32"
        out[key] = {"elements_per_s": m.n_cells * steps / total_s, "ms_per_step": total_s / steps * 1e3,
                    "assemble_avg_ms": a * 1e3, "assemble_stage_ms": statistics.mean(asm_ms),
                    "evaluate_avg_ms": statistics.mean(ev_ms),
                    "assemble_achieved_GBs": asm_bytes / a / 1e9,
                    "assemble_frac": asm_bytes / a / 1e9 / HBM_PEAK_GBS,
                    "step_frac": (asm_bytes + ev_bytes) / (total_s / steps) / 1e9 / HBM_PEAK_GBS}
        if prec != api.FP64 and api.FP64 in states:
            out[key].update(precision_error(pat, states[api.FP64], st))
    for st in states.values():
        st.bc.close()
    out["jacobian_path"] = jacobian_path(stats)
    out["assemble_algorithmic_bytes"] = asm_bytes
    out["evaluate_algorithmic_bytes"] = ev_bytes
    return out


def precision_error(pat, ref, st):
    """The FP32 form against the FP64 form of the same step (the last outputs
    of each): K row-scaled, dc scaled by max |dc|, c relative."""
    import torch
    rp, _ = pat.pattern()
    rows = torch.repeat_interleave(torch.arange(pat.ndof, device="cuda"),
                                   torch.from_numpy(np.diff(rp).astype(np.int64)).cuda())
    torch.cuda.synchronize()
    # every buffer holds the same step's result (the inputs do not change)
    k_err = row_scaled_err(rows, st.Ks[0], ref.Ks[0])
    dc64, dc32 = ref.dcs[0], st.dcs[0].double()
    dc_err = float((dc32 - dc64).abs().max() / dc64.abs().max())
    c_err = float((st.cs[0][0] - ref.cs[0][0]).abs() / ref.cs[0][0].abs())
    return {"K_row_scaled_err_vs_fp64": k_err, "dc_err_vs_fp64": dc_err, "c_rel_err_vs_fp64": c_err}


def jacobian_path(stats):
    """Which contraction the assembly ran: groups of axis-aligned elements
    (diagonal J^-1) use the shorter one, the others the general affine one."""
    d, g = stats["n_groups_diag"], stats["n_groups"]
    kind = "axis-aligned (diagonal J^-1)" if d == g else "general affine (full J^-1)" if d == 0 else "mixed"
    return {"kind": kind, "groups_diagonal": d, "groups": g}


def cpu_info():
    """The host CPU as /proc/cpuinfo names it, its current clock and the
    cores this process may use."""
    model, mhz = platform.processor() or platform.machine(), None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                k, _, v = line.partition(":")
                k = k.strip()
                if k == "model name" and model in ("", "x86_64", platform.machine()):
                    model = v.strip()
                elif k == "cpu MHz" and mhz is None:
                    mhz = float(v)
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "mhz": mhz, "nproc": usable, "cpu_count": os.cpu_count()}


def cpu_baseline_run(passes=5):
    """The CPU oracle on a bounded sample of the headline workload: the same
    cantilever cut to 120 x 40 x 8 elements (38,400 of the 192,000; rho and u
    drawn the same way), one pass = oracle assemble (FP64, full pattern,
    Dirichlet) + sensitivity + compliance; median of `passes` passes, serial
    and as the row-block OpenMP variant (bitwise the serial result)."""
    from oracle import oracle as O
    from paper_2505_02438_amd import inputs as I
    pr = I.cantilever_hex(120, 40, 8)
    m = pr.mesh
    rp, ci = O.pattern(m.elem, m.n_nodes, m.cells)
    res = {}
    for mt in (False, True):
        ts = []
        for _ in range(passes):
            t0 = time.perf_counter()
            O.assemble(m.elem, m.coords, m.cells, pr.rho, rp, ci, mask=pr.mask, mt=mt)
            O.sensitivity(m.elem, m.coords, m.cells, pr.rho, pr.u, mt=mt)
            O.compliance(m.elem, m.coords, m.cells, pr.rho, pr.u, mt=mt)
            ts.append(time.perf_counter() - t0)
        res[mt] = (m.n_cells / statistics.median(ts), ts)
    threads = O.threads()
    hw = cpu_info()
    v1, t1 = res[False]
    vt, tt = res[True]
    return {
        "value": v1, "unit": "elements/s", "cores": 1, "kind": "oracle",
        "sample": f"120x40x8 slab of the same cantilever ({m.n_cells} elements, Q1 hex, rho~Beta(2,2), "
                  f"x=0 clamped); one pass = oracle assemble (FP64, full pattern, Dirichlet) + sensitivity + "
                  f"compliance; median of {passes} passes ({statistics.median(t1):.2f} s), single thread",
        "cpu": hw,
        "row_block_openmp": {"value": vt, "unit": "elements/s", "cores": threads, "kind": "oracle (OpenMP rows)",
                             "median_pass_s": statistics.median(tt), "passes": passes,
                             "speedup_vs_serial": vt / v1},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-passes", type=int, default=5, help="oracle passes of the CPU baseline (median)")
    ap.add_argument("--spin-up", type=float, default=0.3,
                    help="seconds of untimed steps before the warm-up steps (GPU clocks ramp-up)")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the second timed region (the same step replayed as a captured HIP graph)")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="hex120x40x40")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 form of the headline step")
    ap.add_argument("--no-labelled", action="store_true",
                    help="skip the labelled rows (sheared hexahedra, the other workloads)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-solve", action="store_true", help="skip the SpMV / preconditioned CG measurement")
    ap.add_argument("--solve-rtol", type=float, default=1e-9)
    ap.add_argument("--no-filter", action="store_true", help="skip the filter-step measurement")
    ap.add_argument("--no-oc", action="store_true", help="skip the OC-update measurement")
    ap.add_argument("--no-hex27", action="store_true",
                    help="skip the Q2 hexahedron assembly and evaluation (curved 60x20x20 cantilever)")
    ap.add_argument("--no-general", action="store_true",
                    help="skip the per-quadrature-point assembly on general hexahedra")
    ap.add_argument("--no-paper-runs", action="store_true",
                    help="skip the whole optimisation runs of the paper's examples")
    ap.add_argument("--to-iters", type=int, default=3,
                    help="whole optimisation iterations on the 120x40x8 cantilever (0 = skip; the paper ran 155)")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU: the hot path is measured on one "
                                   "GPU's share; multi-GPU sharding is design-only", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_2505_02438_amd import api
    from paper_2505_02438_amd import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    desc, make = WORKLOADS[args.workload]
    pr = make(I)
    m = pr.mesh
    t0 = time.perf_counter()
    pat = api.Pattern.from_mesh(m)
    build_s = time.perf_counter() - t0
    stats = pat.stats()

    stream = torch.cuda.Stream()
    st = StepState(pr, pat, api.FP64, stream)
    mat, rho = st.mat, st.rho

    spun = spin_up(st, stream, args.spin_up)
    total_s, asm_ms, ev_ms = timed_steps(st, stream, args.steps, args.warmup)
    asm_kernel_ms = st.asm_kernel_ms
    graph_s = None
    graphs = None
    if not args.no_graph:
        # HIP graph replay of the eager timed region's step (the same kernels
        # in the same order), captured and timed after the eager region:
        # eager steps timed while captured graphs were held ran slower on
        # some runs (108 vs 90 us assembly)
        # one graph holds one step per output buffer, so a replay runs nbuf
        # steps and its launch cost is shared among them
        graphs = []
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            for b in range(st.nbuf):
                st.fused(b, stream)
        graphs.append(g)
        torch.cuda.synchronize()
    graph_steps = 0
    if graphs is not None:
        with torch.cuda.stream(stream):
            for i in range(max(1, args.warmup // st.nbuf)):
                graphs[0].replay()
        torch.cuda.synchronize()
        reps = max(1, -(-args.steps // st.nbuf))
        graph_steps = reps * st.nbuf
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            for i in range(reps):
                graphs[0].replay()
        torch.cuda.synchronize()
        graph_s = time.perf_counter() - t0
        del graphs  # the captured graphs' memory goes before the other legs

    if args.copy_probe:
        # known traffic for the counter calibration: a 1 GiB fill (writes
        # 1 GiB) and 1 GiB -> 1 GiB elementwise kernels (read 1 GiB, write 1 GiB)
        with torch.cuda.stream(stream):
            x = torch.empty(1 << 27, dtype=torch.float64, device=dev)
            y = torch.empty_like(x)
            x.fill_(1.0)
            for _ in range(3):
                torch.mul(x, 2.0, out=y)
        torch.cuda.synchronize()
        del x, y

    # the box's own streaming rates, for the roofline: a 1 GiB fill (writes)
    # and a 1 GiB copy (reads + writes), HIP events on the bench stream, median
    # of 10 after 2 warm-ups
    def stream_rate(fn, nbytes):
        t = []
        for r in range(12):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            with torch.cuda.stream(stream):
                fn()
            b.record(stream)
            torch.cuda.synchronize()
            if r >= 2:
                t.append(a.elapsed_time(b) / 1e3)
        return nbytes / statistics.median(t) / 1e9
    with torch.cuda.stream(stream):
        sx = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        sy = torch.empty_like(sx)
    torch.cuda.synchronize()
    fill_gbs = stream_rate(lambda: sx.fill_(1.0), 1 << 30)
    copy_gbs = stream_rate(lambda: sy.copy_(sx), 2 << 30)
    del sx, sy

    n = pat.n_cells
    asm_bytes, ev_bytes = algorithmic_bytes(m.n_nodes, n, pat.nnz, m.dim, m.nen, m.ndof)
    # the assembly kernel's average launch: the smaller of the back-to-back
    # bursts and the stage-split region's events around each call
    asm_avg_s = asm_kernel_ms / 1e3
    achieved = asm_bytes / asm_avg_s / 1e9
    step_unique = (pat.nnz * 8 + n * 8 + n * 8 + pat.ndof * 8 + m.n_nodes * m.dim * 8 + n * m.nen * 4 + pat.ndof)
    traffic = None
    if args.workload == "hex120x40x40" and os.path.exists(COUNTERS):
        with open(COUNTERS) as fh:
            cnt = json.load(fh)
        if cnt.get("kernels_hip_sha256_16") == kernel_source_hash():
            traffic = cnt.get("hbm_bytes_per_launch")

    out = {
        "metric": METRIC,
        "value": n * args.steps / total_s,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_s / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": desc + STEP,
            "elements": n, "ndof": pat.ndof, "nnz": pat.nnz, "precision": "fp64",
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_assemble<%d,%d,fp64> with the bound Dirichlet table" % (m.dim, m.nen),
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": asm_bytes,
            "avg_launch_ms": asm_avg_s * 1e3,
            "avg_launch_ms_how": ("the smaller of: the fastest of three bursts of %d assembly-only launches back to back between two HIP events "
             "on the bench stream (%.4f ms); the median of the stage-split region's events around each assembly call "
             "(%.4f ms)") % (args.steps, st.asm_burst_ms, st.asm_each_ms),
            "measured_fill_GBs": fill_gbs,
            "measured_copy_GBs": copy_gbs,
            "frac_of_measured_fill": achieved / fill_gbs,
        },
        "step_frac": (asm_bytes + ev_bytes) / (total_s / args.steps) / 1e9 / HBM_PEAK_GBS,
        # the step's bytes with the inputs both kernels read (rho, coordinates,
        # cells) counted once: K and dc written; rho, u, coordinates, cells
        # and the fixed-dof mask read
        "step_unique_bytes": step_unique,
        "step_frac_unique_bytes": step_unique / (total_s / args.steps) / 1e9 / HBM_PEAK_GBS,
        "stage_ms": {"assemble_dirichlet": statistics.mean(asm_ms), "evaluate": statistics.mean(ev_ms)},
        "stage_ms_pct": {"assemble_dirichlet": pct(asm_ms), "evaluate": pct(ev_ms)},
        "launch": ("eager; value and ms_per_step: the timed region, one soptx_step call per step (energies, then "
                   "the assembly, which adds the partials of c), no events between steps; stage_ms: the "
                   "stage-split region right after it, the same steps as two calls (soptx_step for K, "
                   "soptx_evaluate for dc and c) with HIP events around each; roofline: the assembly alone, "
                   "launched back to back between two events"),
        "spin_up": {"seconds": args.spin_up, "steps": spun,
                    "note": "untimed steps before the warm-up steps, so that the GPU clocks have ramped"},
        "jacobian_path": jacobian_path(stats),
        "graph_value": None if graph_s is None else n * graph_steps / graph_s,
        "graph_ms_per_step": None if graph_s is None else graph_s / graph_steps * 1e3,
        "graph_steps": graph_steps,
        "evaluate_algorithmic_bytes": ev_bytes,
        "pattern_build_s": build_s,
        "plan": {"groups": stats["n_groups"], "signatures": stats["n_signatures"],
                 "plan_bytes": stats["plan_bytes"]},
    }
    if not args.no_fp32:
        st32 = StepState(pr, pat, api.FP32, stream)
        spin_up(st32, stream, 0.2)
        t32, a32, e32 = timed_steps(st32, stream, args.steps, args.warmup)
        out["fp32"] = {"value": n * args.steps / t32, "ms_per_step": t32 / args.steps * 1e3,
                       "stage_ms": {"assemble_dirichlet": statistics.mean(a32), "evaluate": statistics.mean(e32)},
                       "value_ratio_vs_fp64": (n * args.steps / t32) / out["value"]}
        out["fp32"].update(precision_error(pat, st, st32))
        st32.bc.close()
        del st32
    if not args.no_solve:
        f = torch.from_numpy(pr.f).to(dev)
        out["solve"] = solve_run(pat, m, st.Ks[0], f, stream, args.solve_rtol)
    if not args.no_filter:
        out["filter"] = filter_run(pat, m, mat, rho, st.Ks[0], stream)
    if not args.no_oc:
        out["oc"] = oc_run(pat, pat.n_cells, st.dcs[0], stream)
    st.bc.close()
    del st
    torch.cuda.empty_cache()
    if not args.no_labelled:
        rows = {}
        for wl in ("hex120x40x40_sheared", "hex120x40x40_renumbered", "tri600x200", "p2box48"):
            if wl != args.workload:
                d, mk = WORKLOADS[wl]
                rows[wl] = labelled_run(wl, d, mk(I), stream, min(args.steps, 20), 3,
                                        (api.FP64, api.FP32) if wl in ("p2box48", "tri600x200") else (api.FP64,))
                torch.cuda.empty_cache()
        out["labelled"] = rows
    if args.to_iters > 0:
        out["optimisation_loop"] = to_loop_run(args.to_iters, stream)
    if not args.no_general:
        out["general_assembly"] = general_run(stream)
        out["general_assembly_2d"] = general_run(stream, two_d=True)
    if not args.no_hex27:
        out["hex27_assembly"] = hex27_run(stream)
    if not args.no_paper_runs:
        out["paper_runs"] = paper_runs()
    if not args.no_serving:
        out["serving"] = serving_run(args.serve_requests)
        out["serving"]["burst_vs_plain"] = out["serving"]["burst_elements_per_s"] / out["value"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_run(args.cpu_passes)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
