"""Assembly with per-quadrature-point geometry (soptx_assemble_general) on
the GPU, through the C ABI: general (non-affine) Q1 quadrilaterals and
hexahedra against the oracle's assembly (row-scaled error, the C12 metric,
<= 1e-12), with and without Dirichlet rows; the three forms of the assembly
(in LDS on the plan's node groups with the block sums in registers or in an
LDS stage, and through element matrices in memory) against the oracle and
each other, also on renumbered meshes; a mesh with more work items per node
group than the register form holds takes the stage form; on affine meshes
against the separated-form kernel (two different formulas, same matrix);
determinism; the affine-only calls refuse a non-affine handle; the full
120x40x40 hexahedral cantilever with jittered interior nodes against the
oracle."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2505_02438_amd import _lib, api
from paper_2505_02438_amd import inputs as I

from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _row_scaled(rp, Kg, Kr):
    n = len(rp) - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    den = np.zeros(n)
    np.maximum.at(den, rows, np.abs(Kr))
    num = np.zeros(n)
    np.maximum.at(num, rows, np.abs(Kg - Kr))
    return float(np.max(num / np.where(den > 0, den, 1.0)))


def _jittered(elem, dims, amount, seed):
    rng = np.random.default_rng(seed)
    m0 = I.quad_grid(*dims) if elem == I.QUAD4 else I.hex_grid(*dims)
    return I.jitter_interior(m0, amount, rng), rng


@pytest.mark.parametrize("elem,dims", [(I.QUAD4, (9, 7)), (I.QUAD4, (33, 17)), (I.HEX8, (5, 4, 3)),
                                       (I.HEX8, (11, 6, 5))])
def test_general_matches_oracle(elem, dims):
    m, rng = _jittered(elem, dims, 0.3, 51)
    pat = api.Pattern.from_mesh(m, general=True)
    rho = rng.uniform(1e-3, 1.0, m.n_cells)
    mat = api.Material(E0=1.0, Emin=1e-9, nu=0.3, p=3.0)
    rp, ci = O.pattern(elem, m.n_nodes, m.cells)
    mask = (rng.uniform(size=m.ndof) < 0.1).astype(np.uint8)
    for msk in (None, mask):
        K = host(pat.assemble_general(mat, dev(rho), None if msk is None else dev(msk)))
        Kr = O.assemble(elem, m.coords, m.cells, rho, rp, ci, mask=msk)
        err = _row_scaled(rp, K, Kr)
        print(f"elem={elem} {dims} mask={msk is not None}: row-scaled {err:.1e}")
        assert err <= 1e-12
        if msk is not None:
            # Dirichlet rows and columns exactly as the oracle sets them
            fixed = np.nonzero(msk)[0]
            rows = np.repeat(np.arange(m.ndof), np.diff(rp))
            sel = np.isin(rows, fixed) | np.isin(ci, fixed)
            assert np.array_equal(K[sel], Kr[sel])


def _in_lds(pat):
    v = ctypes.c_int32(-1)
    assert _lib.lib().soptx_debug_general_path(pat._h, ctypes.byref(v)) == 0
    return v.value


def _renumbered(m, rng):
    pn, pe = rng.permutation(m.n_nodes), rng.permutation(m.n_cells)
    coords = np.empty_like(m.coords)
    coords[pn] = m.coords
    return I.Mesh(m.elem, coords, pn[m.cells[pe]].astype(np.int32))


@pytest.mark.parametrize("elem,dims,jit,renum", [(I.QUAD4, (9, 7), 0.3, False), (I.QUAD4, (40, 13), 0.3, True),
                                                 (I.HEX8, (5, 4, 3), 0.3, False), (I.HEX8, (13, 6, 5), 0.3, False),
                                                 (I.HEX8, (9, 7, 5), 0.2, True), (I.HEX8, (9, 7, 5), 0.3, True)])
def test_general_forms_match_oracle_and_each_other(elem, dims, jit, renum):
    """The in-LDS forms (one workgroup per node group of the plan, the
    Jacobian at every Gauss point of each element slot; the blocks' sums in
    registers or in an LDS stage) and the element-matrix form: each against
    the oracle, and against each other
    (the same contributions in the same element order, different rounding
    of the per-point products); renumbered meshes take a canonical-order
    plan (the quadrilaterals and the hexahedra jittered by 0.2 here), the
    others a plan in their own numbering."""
    m, rng = _jittered(elem, dims, jit, 55)
    if renum:
        m = _renumbered(m, rng)
    pat = api.Pattern.from_mesh(m, general=True)
    rho = rng.uniform(1e-3, 1.0, m.n_cells)
    mat = api.Material(E0=1.0, Emin=1e-9, nu=0.3, p=3.0)
    rp, ci = O.pattern(elem, m.n_nodes, m.cells)
    Kr = O.assemble(elem, m.coords, m.cells, rho, rp, ci)
    L = _lib.lib()
    assert L.soptx_debug_set_general_variant(2) == -1
    out = {}
    mask = (rng.uniform(size=m.ndof) < 0.1).astype(np.uint8)
    Krm = O.assemble(elem, m.coords, m.cells, rho, rp, ci, mask=mask)
    rows = np.repeat(np.arange(m.ndof), np.diff(rp))
    fixed = np.nonzero(mask)[0]
    sel = np.isin(rows, fixed) | np.isin(ci, fixed)
    try:
        for v in (-1, 1, 0):
            assert L.soptx_debug_set_general_variant(v) == 0
            out[v] = (host(pat.assemble_general(mat, dev(rho))), _in_lds(pat),
                      host(pat.assemble_general(mat, dev(rho), dev(mask))))
    finally:
        L.soptx_debug_set_general_variant(-1)
    # forms: 1 sums in registers, 2 sums in the LDS stage, 0 element matrices
    assert out[-1][1] == 1 and out[1][1] == 2 and out[0][1] == 0
    e = {v: _row_scaled(rp, out[v][0], Kr) for v in out}
    e_mut = max(_row_scaled(rp, out[-1][0], out[v][0]) for v in (1, 0))
    print(f"elem={elem} {dims} jitter {jit} renumbered={renum}: in LDS, sums in registers {e[-1]:.1e}, "
          f"in the stage {e[1]:.1e}; element matrices {e[0]:.1e}; between {e_mut:.1e}")
    assert max(e.values()) <= 1e-12 and e_mut <= 1e-13
    for v in out:
        # with Dirichlet rows: the fixed rows and columns exactly the oracle's,
        # the rest as without
        Km = out[v][2]
        assert np.array_equal(Km[sel], Krm[sel]), v
        assert np.array_equal(Km[~sel], out[v][0][~sel]), v


@pytest.mark.parametrize("case", ["quad_unit", "hex_unit", "quad_sheared", "hex_sheared"])
def test_general_equals_separated_form_on_affine_meshes(case):
    elem = I.QUAD4 if case.startswith("quad") else I.HEX8
    m = I.quad_grid(12, 7) if elem == I.QUAD4 else I.hex_grid(6, 5, 4)
    if case.endswith("sheared"):
        m = I.skew_mesh(m, "global")
    rng = np.random.default_rng(52)
    rho = dev(rng.uniform(1e-3, 1.0, m.n_cells))
    mat = api.Material(E0=1.0, Emin=1e-9, nu=0.3, p=3.0)
    pg = api.Pattern.from_mesh(m, general=True)
    pa = api.Pattern.from_mesh(m)
    Kg, Ka = host(pg.assemble_general(mat, rho)), host(pa.assemble(mat, rho))
    rp, _ = pa.pattern()
    err = _row_scaled(rp, Kg, Ka)
    print(f"{case}: per-point vs separated form, row-scaled {err:.1e}")
    assert err <= 1e-13
    # an affine mesh built for the general path still runs the affine-only calls
    dc, c = pg.evaluate(mat, rho, dev(rng.standard_normal(m.ndof)))
    assert torch.isfinite(c).all()


def test_general_deterministic_and_refusals():
    m, rng = _jittered(I.HEX8, (6, 4, 4), 0.25, 53)
    pat = api.Pattern.from_mesh(m, general=True)
    mat = api.Material()
    rho = dev(rng.uniform(0.01, 1.0, m.n_cells))
    assert torch.equal(pat.assemble_general(mat, rho), pat.assemble_general(mat, rho))
    u = dev(rng.standard_normal(m.ndof))
    for call in (lambda: pat.assemble(mat, rho), lambda: pat.evaluate(mat, rho, u),
                 lambda: pat.sensitivity(mat, rho, u)):
        with pytest.raises(_lib.SoptxError) as e:
            call()
        assert e.value.code == -5
    # the solve works on any handle
    mask, f = I.clamp_x0_bc(m)
    K = pat.assemble_general(mat, rho, dev(mask))
    x, it, rel = pat.pcg(K, dev(f), rtol=1e-10)
    r = dev(f) - pat.spmv(K, x)
    assert float(torch.linalg.norm(r) / torch.linalg.norm(dev(f))) <= 1e-9
    # a pattern built by the affine-only build refuses the general assembly
    pa = api.Pattern.from_mesh(I.hex_grid(3, 3, 3))
    with pytest.raises(_lib.SoptxError) as e:
        pa.assemble_general(mat, dev(np.full(27, 0.5)))
    assert e.value.code == -1


def test_general_full_cantilever_hex():
    """The 3D cantilever's 120 x 40 x 40 hexahedra with every interior node
    moved by up to 0.2: the whole matrix against the oracle."""
    pr = I.cantilever_hex()
    m = I.jitter_interior(pr.mesh, 0.2, np.random.default_rng(54))
    pat = api.Pattern.from_mesh(m, general=True)
    assert _in_lds(pat) == 1  # sums in registers
    mat = api.Material(E0=pr.E0, Emin=pr.Emin, nu=pr.nu, p=pr.p)
    K = host(pat.assemble_general(mat, dev(pr.rho), dev(pr.mask)))
    rp, ci = O.pattern(m.elem, m.n_nodes, m.cells)
    Kr = O.assemble(m.elem, m.coords, m.cells, pr.rho, rp, ci, mask=pr.mask)
    err = _row_scaled(rp, K, Kr)
    print(f"full 120x40x40 jittered hex: row-scaled {err:.1e}")
    assert err <= 1e-12


def _scaled_dc(m, rho, u, dc_gpu, dc_ref, p=3.0, E0=1.0, Emin=1e-9):
    """|dc - dc_ref| / (|E'| |u_e|^T |K_e^0| |u_e|) per element (the condition-scaled metric)."""
    dE = p * rho ** (p - 1) * (E0 - Emin)
    scale = np.empty(m.n_cells)
    uu = u.reshape(-1, m.dim)
    for e in range(m.n_cells):
        Ke = O.element_ke0(m.elem, m.coords[m.cells[e]])
        ue = np.abs(uu[m.cells[e]].ravel())
        scale[e] = dE[e] * (ue @ np.abs(Ke) @ ue)
    return float(np.max(np.abs(dc_gpu - dc_ref) / scale))


@pytest.mark.parametrize("elem,dims", [(I.QUAD4, (9, 7)), (I.HEX8, (5, 4, 3))])
def test_evaluate_general_matches_oracle(elem, dims):
    m, rng = _jittered(elem, dims, 0.3, 55)
    pat = api.Pattern.from_mesh(m, general=True)
    rho = rng.uniform(1e-3, 1.0, m.n_cells)
    u = rng.standard_normal(m.ndof)
    f = rng.standard_normal(m.ndof)
    mat = api.Material(E0=1.0, Emin=1e-9, nu=0.3, p=3.0)
    dc, c = pat.evaluate_general(mat, dev(rho), dev(u), f=dev(f))
    dc, c = host(dc), host(c)
    dref = O.sensitivity(elem, m.coords, m.cells, rho, u)
    cref = O.compliance(elem, m.coords, m.cells, rho, u, f)
    err = _scaled_dc(m, rho, u, dc, dref)
    E = 1e-9 + rho ** 3 * (1 - 1e-9)
    cscale = float(np.sum(E * np.abs(dref) / (3 * rho ** 2 * (1 - 1e-9))))
    print(f"elem={elem} {dims}: dc scaled {err:.1e}, c {abs(c[0] - cref[0]) / cscale:.1e}, f.u {c[1]} / {cref[1]}")
    assert err <= 1e-12 and abs(c[0] - cref[0]) <= 1e-12 * cscale
    assert abs(c[1] - cref[1]) <= 1e-13 * float(np.abs(f) @ np.abs(u))
    # on an affine mesh the same as the separated-form kernels
    ma = I.hex_grid(4, 3, 3) if elem == I.HEX8 else I.quad_grid(7, 5)
    pg, pa = api.Pattern.from_mesh(ma, general=True), api.Pattern.from_mesh(ma)
    ra, ua = dev(rng.uniform(0.01, 1, ma.n_cells)), dev(rng.standard_normal(ma.ndof))
    dg, cg = pg.evaluate_general(mat, ra, ua)
    da, ca = pa.evaluate(mat, ra, ua)
    assert float(torch.max(torch.abs(dg - da) / torch.abs(da))) <= 1e-12
    assert abs(float(cg[0] - ca[0])) <= 1e-13 * abs(float(ca[0]))


def test_general_optimisation_iterations_match_oracle():
    """Five iterations of Algorithm 1 on a jittered 60 x 20 MBB beam, all on the
    GPU with the per-point geometry, against the same iterations of the oracles."""
    from oracle import filters as OF
    from oracle import oc as OC
    from paper_2505_02438_amd import loop
    m = I.jitter_interior(I.quad_grid(60, 20), 0.2, np.random.default_rng(56))
    mask, f = I.mbb_bc(m)
    res = loop.run(m, mask, f, 0.5, 1.5, max_iter=5, tol=0.0, cg_rtol=1e-12, general=True)
    rp, ci = O.pattern(m.elem, m.n_nodes, m.cells)
    cent = OF.centroids(m.elem, m.coords, m.cells)
    H = OF.filter_matrix(cent, 1.5)
    v = OF.volumes(m.elem, m.coords, m.cells)
    rho = np.full(m.n_cells, 0.5)
    for it in range(5):
        K = O.assemble(m.elem, m.coords, m.cells, rho, rp, ci, mask=mask)
        uo = O.solve(rp, ci, K, f)
        co = O.compliance(m.elem, m.coords, m.cells, rho, uo, f)[1]
        dco = O.sensitivity(m.elem, m.coords, m.cells, rho, uo)
        rho, *_ = OC.oc_update(rho, OF.sensitivity_filter(H, rho, dco), v, 0.5 * v.sum(), move=0.2, eta=0.5)
        print(f"iteration {it}: c {res.compliance[it]:.10f} / {co:.10f}")
        assert abs(res.compliance[it] - co) <= 1e-8 * co
    assert float(np.max(np.abs(host(res.rho) - rho))) <= 1e-6


def _quad_star(n, rng):
    """n kite-shaped quadrilaterals around one centre node (centre, p_k, o_k,
    p_k+1 counter-clockwise; p on the unit circle, o at radius 2 between),
    the ring nodes jittered: none is a parallelogram, and the centre has
    2 n + 1 neighbours."""
    c = np.zeros((1, 2))
    t = 2 * np.pi * np.arange(n) / n
    p = np.stack([np.cos(t), np.sin(t)], 1) * (1 + rng.uniform(-0.05, 0.05, (n, 1)))
    o = 2 * np.stack([np.cos(t + np.pi / n), np.sin(t + np.pi / n)], 1) * (1 + rng.uniform(-0.05, 0.05, (n, 1)))
    coords = np.concatenate([c, p, o])
    cells = np.array([[0, 1 + k, 1 + n + k, 1 + (k + 1) % n] for k in range(n)], dtype=np.int32)
    return I.Mesh(I.QUAD4, coords, cells)


def test_general_many_work_items_take_the_stage_form():
    """A node with 21 neighbours gives its group more work items than the
    register form holds (two per wave): the default then runs the stage form,
    which matches the oracle; the element-matrix form agrees."""
    rng = np.random.default_rng(56)
    m = _quad_star(10, rng)
    pat = api.Pattern.from_mesh(m, general=True)
    rho = rng.uniform(1e-3, 1.0, m.n_cells)
    mat = api.Material(E0=1.0, Emin=1e-9, nu=0.3, p=3.0)
    rp, ci = O.pattern(m.elem, m.n_nodes, m.cells)
    Kr = O.assemble(m.elem, m.coords, m.cells, rho, rp, ci)
    assert _in_lds(pat) == 2
    K = host(pat.assemble_general(mat, dev(rho)))
    L = _lib.lib()
    try:
        assert L.soptx_debug_set_general_variant(0) == 0
        assert _in_lds(pat) == 0
        Ke = host(pat.assemble_general(mat, dev(rho)))
    finally:
        L.soptx_debug_set_general_variant(-1)
    e, e_mut = _row_scaled(rp, K, Kr), _row_scaled(rp, K, Ke)
    print(f"star of 10 quadrilaterals: stage form {e:.1e}, against element matrices {e_mut:.1e}")
    assert e <= 1e-12 and e_mut <= 1e-13
