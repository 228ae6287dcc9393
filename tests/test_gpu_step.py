"""The fused step (soptx_step: assembly with a bound Dirichlet table applied
while the blocks are staged, then element energies, dc and c) through the C
ABI:

* against the separate calls on the same inputs: K bit for bit equal to
  soptx_assemble with the mask, dc and c bit for bit equal to soptx_evaluate
  (the same kernels), in both precision forms;
* against the oracle at the parity tolerances (row-scaled K, condition-scaled
  dc, c), in both precision forms, on all element types, with several groups
  per signature, ragged last groups and general (sheared) Q1 maps;
* the optional outputs (no u, no dc, no c, no f), an empty mask, run-to-run
  bitwise reproducibility, and argument errors before any device work."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2505_02438_amd import _lib, api
from paper_2505_02438_amd import inputs as I

from gpu_util import E, abs_energy, dE, dev, host, row_scaled_err

pytestmark = pytest.mark.gpu
ELEMS = [I.QUAD4, I.TRI3, I.HEX8, I.TET10]
MAT = api.Material()
TOL = {api.FP64: 1e-12, api.FP32: 1e-5}
CASES = ([(e, None, None) for e in ELEMS] + [(I.QUAD4, (23, 9), "global"), (I.HEX8, (9, 6, 7), "global"),
         (I.HEX8, (9, 6, 7), "kink"), (I.HEX8, (13, 4, 37), None), (I.TET10, (4, 3, 3), None),
         (I.TRI3, (31, 12), None)] + [(e, d, "renumbered") for e, d in
                                      ((I.QUAD4, (23, 9)), (I.TRI3, (31, 12)), (I.HEX8, (9, 6, 7)), (I.TET10, (4, 3, 3)))])


def _setup(elem, dims, skew, seed=7):
    pr = I.small_problem(elem, seed=seed, dims=dims, skew=None if skew == "renumbered" else skew)
    if skew == "renumbered":
        pr = I.renumber(pr, seed + 100)
    m = pr.mesh
    pat = api.Pattern(elem, m.coords, m.cells)
    if skew == "renumbered":
        assert pat.stats()["n_groups_ranked"] > 0
    rp, ci = O.pattern(elem, m.n_nodes, m.cells)
    return pr, m, pat, rp, ci


@pytest.mark.parametrize("elem,dims,skew", CASES)
def test_step_fp64_equals_separate_calls_and_oracle(elem, dims, skew):
    pr, m, pat, rp, ci = _setup(elem, dims, skew)
    bc = api.Dirichlet(pat, pr.mask)
    assert bc.n_fixed == int(np.count_nonzero(pr.mask)) and bc.n_groups > 0
    rho, u, f = dev(pr.rho), dev(pr.u), dev(pr.f)
    K, dc, c = pat.step(MAT, rho, u, f, bc=bc)
    torch.cuda.synchronize()
    K, dc, c = host(K), host(dc), host(c)
    # the separate calls
    Ks = host(pat.assemble(MAT, rho, dev(pr.mask)))
    dcs, cs = pat.evaluate(MAT, rho, u, f)
    dcs, cs = host(dcs), host(cs)
    assert np.array_equal(K, Ks), "K differs from soptx_assemble + Dirichlet"
    assert np.array_equal(dc, dcs) and np.array_equal(c, cs), "dc or c differ from soptx_evaluate"
    # the oracle
    Kref = O.assemble(elem, m.coords, m.cells, pr.rho, rp, ci, mask=pr.mask)
    dref = O.sensitivity(elem, m.coords, m.cells, pr.rho, pr.u)
    cref = O.compliance(elem, m.coords, m.cells, pr.rho, pr.u, pr.f)
    scale = abs_energy(m, pr.u, np.arange(m.n_cells))
    kerr = row_scaled_err(rp, K, Kref)
    derr = np.max(np.abs(dc - dref) / (dE(pr.rho) * scale))
    cerr = abs(c[0] - cref[0]) / np.sum(E(pr.rho) * scale)
    print(f"elem={elem} dims={dims} skew={skew} groups={pat.stats()['n_groups']} touched={bc.n_groups} "
          f"K {kerr:.1e} dc {derr:.1e} c {cerr:.1e}")
    assert kerr <= TOL[api.FP64] and derr <= TOL[api.FP64] and cerr <= TOL[api.FP64]
    assert abs(c[1] - cref[1]) <= 1e-14 * np.sum(np.abs(pr.f * pr.u))
    bc.close()


@pytest.mark.parametrize("elem", ELEMS)
def test_step_fp32(elem):
    pr, m, pat, rp, ci = _setup(elem, None, None)
    bc = api.Dirichlet(pat, pr.mask)
    rho32 = dev(pr.rho, torch.float32)
    K, dc, c = pat.step(MAT, rho32, dev(pr.u), bc=bc, prec=api.FP32)
    Ks = pat.assemble(MAT, rho32, dev(pr.mask), prec=api.FP32)
    dcs, cs = pat.evaluate(MAT, rho32, dev(pr.u), prec=api.FP32)
    torch.cuda.synchronize()
    assert dc.dtype == torch.float32
    assert np.array_equal(host(K), host(Ks))
    assert np.array_equal(host(dc), host(dcs)) and np.array_equal(host(c), host(cs))
    rho_r = pr.rho.astype(np.float32).astype(np.float64)
    dref = O.sensitivity(elem, m.coords, m.cells, rho_r, pr.u)
    cref = O.compliance(elem, m.coords, m.cells, rho_r, pr.u)
    scale = abs_energy(m, pr.u, np.arange(m.n_cells))
    derr = np.max(np.abs(host(dc).astype(np.float64) - dref) / (dE(rho_r) * scale))
    cerr = abs(host(c)[0] - cref[0]) / np.sum(E(rho_r) * scale)
    Kref = O.assemble(elem, m.coords, m.cells, rho_r, rp, ci, mask=pr.mask)
    kerr = row_scaled_err(rp, host(K), Kref)
    print(f"elem={elem} FP32 step: K {kerr:.1e} dc {derr:.1e} c {cerr:.1e}")
    assert kerr <= TOL[api.FP32] and derr <= TOL[api.FP32] and cerr <= TOL[api.FP32]


@pytest.mark.parametrize("elem", [I.QUAD4, I.HEX8, I.TET10])
def test_step_optional_outputs_and_reproducibility(elem):
    pr, m, pat, rp, ci = _setup(elem, None, None)
    bc = api.Dirichlet(pat, pr.mask)
    rho, u, f = dev(pr.rho), dev(pr.u), dev(pr.f)
    K0, dc0, c0 = (host(t) for t in pat.step(MAT, rho, u, f, bc=bc))
    # run to run
    for _ in range(3):
        K1, dc1, c1 = (host(t) for t in pat.step(MAT, rho, u, f, bc=bc))
        assert np.array_equal(K0, K1) and np.array_equal(dc0, dc1) and np.array_equal(c0, c1)
    # assembly only (no u): K unchanged
    Ka, dca, ca = pat.step(MAT, rho, bc=bc)
    assert dca is None and ca is None and np.array_equal(host(Ka), K0)
    # dc only; c only; no f (c[1] = 0)
    _, dcb, cb = pat.step(MAT, rho, u, bc=bc, want_c=False)
    assert cb is None and np.array_equal(host(dcb), dc0)
    _, dcc, cc = pat.step(MAT, rho, u, f, bc=bc, want_dc=False)
    assert dcc is None and np.array_equal(host(cc), c0)
    _, _, cd = pat.step(MAT, rho, u, bc=bc, want_dc=False)
    assert host(cd)[0] == c0[0] and host(cd)[1] == 0.0
    # no Dirichlet table: soptx_assemble without a mask
    Kn, _, _ = pat.step(MAT, rho, bc=None)
    assert np.array_equal(host(Kn), host(pat.assemble(MAT, rho)))
    # an empty mask: a table that touches no group
    bc0 = api.Dirichlet(pat, np.zeros(m.ndof, np.uint8))
    assert bc0.n_fixed == 0 and bc0.n_groups == 0
    Ke, _, _ = pat.step(MAT, rho, bc=bc0)
    assert np.array_equal(host(Ke), host(Kn))


def test_step_argument_errors():
    pr, m, pat, rp, ci = _setup(I.HEX8, None, None)
    bc = api.Dirichlet(pat, pr.mask)
    other = api.Pattern.from_mesh(I.hex_grid(2, 2, 2))
    bco = api.Dirichlet(other, np.zeros(other.ndof, np.uint8))
    rho, u = dev(pr.rho), dev(pr.u)
    K = torch.full((pat.nnz,), 7.0, dtype=torch.float64, device="cuda")
    dc = torch.full((m.n_cells,), 7.0, dtype=torch.float64, device="cuda")
    L = _lib.lib()
    mc = MAT._c()
    # a table of another pattern; dc without u; bf16; NULL handle
    assert L.soptx_step(pat._h, bco._h, ctypes.byref(mc), rho.data_ptr(), u.data_ptr(), None, K.data_ptr(),
                        dc.data_ptr(), None, 0, None) == -1
    assert L.soptx_step(pat._h, bc._h, ctypes.byref(mc), rho.data_ptr(), None, None, K.data_ptr(),
                        dc.data_ptr(), None, 0, None) == -1
    assert L.soptx_step(pat._h, bc._h, ctypes.byref(mc), rho.data_ptr(), u.data_ptr(), None, K.data_ptr(),
                        dc.data_ptr(), None, 2, None) == -1
    assert L.soptx_step(None, None, ctypes.byref(mc), None, None, None, None, None, None, 0, None) == -1
    torch.cuda.synchronize()
    assert bool((K == 7.0).all()) and bool((dc == 7.0).all())
    with pytest.raises(ValueError):
        api.Dirichlet(pat, np.zeros(3, np.uint8))
    out = ctypes.c_void_p(1)
    assert L.soptx_build_dirichlet(None, None, ctypes.byref(out), None) == -1 and out.value is None


@pytest.mark.parametrize("elem,dims,skew", [(I.QUAD4, (23, 9), None), (I.TRI3, (31, 12), None),
                                            (I.HEX8, (9, 6, 7), "global"), (I.TET10, (4, 3, 3), None),
                                            (I.HEX8, (9, 6, 7), "renumbered"), (I.TRI3, (31, 12), "renumbered")])
def test_assembly_kernels_agree_bitwise(elem, dims, skew):
    """The persistent assembly kernel and the one-workgroup-per-group kernel
    (chosen by the plan's shape; forced here through the debug hook) give
    bitwise the same K, with and without the bound Dirichlet table, in both
    precision forms.  In the fused step with u the assembly kernel also adds
    the energy kernel's partials of c: under either kernel, dc and c are
    bitwise those of soptx_evaluate (k_finalize)."""
    pr, m, pat, rp, ci = _setup(elem, dims, skew)
    bc = api.Dirichlet(pat, pr.mask)
    L = _lib.lib()
    u, f = dev(pr.u), dev(pr.f)
    out, fused = {}, {}
    try:
        for v in (0, 1, -1):
            assert L.soptx_debug_set_assembly_variant(v) == 0
            for prec in (api.FP64, api.FP32):
                rho = dev(pr.rho) if prec == api.FP64 else dev(pr.rho).float()
                K1 = host(pat.assemble(MAT, rho, prec=prec))
                K2, _, _ = pat.step(MAT, rho, bc=bc, prec=prec)
                out[(v, prec)] = (K1, host(K2))
                K3, dc3, c3 = pat.step(MAT, rho, u, f, bc=bc, prec=prec)
                dce, ce = pat.evaluate(MAT, rho, u, f, prec=prec)
                fused[(v, prec)] = (host(K3), host(dc3), host(c3), host(dce), host(ce))
        assert L.soptx_debug_set_assembly_variant(2) == -1
    finally:
        L.soptx_debug_set_assembly_variant(-1)
    for prec in (api.FP64, api.FP32):
        for v in (1, -1):
            assert np.array_equal(out[(v, prec)][0], out[(0, prec)][0]), (v, prec)
            assert np.array_equal(out[(v, prec)][1], out[(0, prec)][1]), (v, prec)
        for v in (0, 1, -1):
            K3, dc3, c3, dce, ce = fused[(v, prec)]
            assert np.array_equal(K3, out[(0, prec)][1]), (v, prec)
            assert np.array_equal(dc3, dce) and np.array_equal(c3, ce), (v, prec, c3, ce)
            assert c3[1] != 0.0


def test_step_degenerate_meshes():
    """The fused step on meshes without work for the assembly: no cells and no
    nodes; nodes but no cells (no groups: the compliance partials are summed
    by their own launch, c = [0, f^T u]); a grid beside an isolated node (the
    assembly kernel sums them).  dc and c equal soptx_evaluate's bit for bit."""
    # no cells, no nodes
    pat = api.Pattern(I.HEX8, np.zeros((0, 3)), np.zeros((0, 8), dtype=np.int32))
    z = torch.zeros(0, dtype=torch.float64, device="cuda:0")
    K, dc, c = pat.step(MAT, z, z, z, K=torch.zeros(0, dtype=torch.float64, device="cuda:0"))
    torch.cuda.synchronize()
    assert host(c)[0] == 0.0 and host(c)[1] == 0.0 and dc.numel() == 0
    # nodes but no cells
    coords = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 2.0, 1.0]])
    pat = api.Pattern(I.HEX8, coords, np.zeros((0, 8), dtype=np.int32))
    assert pat.stats()["n_groups"] == 0
    u = np.linspace(-1.0, 2.0, pat.ndof)
    f = np.cos(np.arange(pat.ndof, dtype=np.float64))
    K, dc, c = pat.step(MAT, z, dev(u), dev(f), K=torch.zeros(pat.nnz, dtype=torch.float64, device="cuda:0"))
    torch.cuda.synchronize()
    c = host(c)
    assert c[0] == 0.0 and abs(c[1] - float(np.dot(f, u))) <= 1e-14 * np.sum(np.abs(f * u))
    # a grid beside an isolated node
    m = I.quad_grid(5, 3)
    coords = np.vstack([m.coords, [[10.0, 10.0]]])
    pat = api.Pattern(I.QUAD4, coords, m.cells)
    assert pat.stats()["n_groups"] > 0
    rho = dev(np.linspace(0.1, 1.0, m.n_cells))
    u = dev(np.sin(np.arange(pat.ndof, dtype=np.float64)))
    f = dev(np.cos(np.arange(pat.ndof, dtype=np.float64)))
    _, dc1, c1 = pat.step(MAT, rho, u, f)
    dc2, c2 = pat.evaluate(MAT, rho, u, f)
    torch.cuda.synchronize()
    assert np.array_equal(host(dc1), host(dc2)) and np.array_equal(host(c1), host(c2))
