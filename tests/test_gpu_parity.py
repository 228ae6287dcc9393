"""GPU parity of the HIP path against the CPU oracle on small meshes (several
groups, ragged last groups, all element types), through the C ABI."""
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


def _setup(elem, seed=7, dims=None, ref=api.REF_SYMBOLIC, skew=None):
    pr = I.small_problem(elem, seed=seed, dims=dims, skew=skew)
    m = pr.mesh
    pat = api.Pattern(elem, m.coords, m.cells, ref_method=ref)
    rp, ci = O.pattern(elem, m.n_nodes, m.cells)
    return pr, m, pat, rp, ci


@pytest.mark.parametrize("elem", ELEMS)
def test_pattern_bit_exact(elem):
    pr, m, pat, rp, ci = _setup(elem)
    drp, dci = pat.pattern()
    assert pat.nnz == ci.size and pat.ndof == m.ndof
    assert np.array_equal(drp.astype(np.int64), rp) and np.array_equal(dci, ci)


@pytest.mark.parametrize("elem", ELEMS)
@pytest.mark.parametrize("use_mask", [False, True])
@pytest.mark.parametrize("ref", [api.REF_SYMBOLIC, api.REF_QUADRATURE])
def test_assemble_fp64(elem, use_mask, ref):
    pr, m, pat, rp, ci = _setup(elem, ref=ref)
    mask = pr.mask if use_mask else None
    K = host(pat.assemble(MAT, dev(pr.rho), None if mask is None else dev(mask)))
    Kref = O.assemble(elem, m.coords, m.cells, pr.rho, rp, ci, mask=mask)
    err = row_scaled_err(rp, K, Kref)
    print(f"elem={elem} mask={use_mask} ref={ref} K row-scaled err {err:.2e}")
    assert err <= TOL[api.FP64]


@pytest.mark.parametrize("elem", ELEMS)
def test_apply_dirichlet_separately(elem):
    """assemble(mask) == assemble() then apply_dirichlet(mask), bit for bit."""
    pr, m, pat, rp, ci = _setup(elem)
    K1 = host(pat.assemble(MAT, dev(pr.rho), dev(pr.mask)))
    K2 = pat.assemble(MAT, dev(pr.rho), None)
    K2 = host(pat.apply_dirichlet(dev(pr.mask), K2))
    assert np.array_equal(K1, K2)


@pytest.mark.parametrize("elem", [I.QUAD4, I.HEX8])
@pytest.mark.parametrize("skew", ["global", "kink"])
@pytest.mark.parametrize("use_mask", [False, True])
def test_assemble_fp64_skewed_q1(elem, skew, use_mask):
    """General-Jacobian groups ('global') and a mix of axis-aligned and general
    groups ('kink') on Q1 meshes, with several groups per signature."""
    pr, m, pat, rp, ci = _setup(elem, skew=skew, dims=(23, 9) if elem == I.QUAD4 else (9, 6, 7))
    mask = pr.mask if use_mask else None
    K = host(pat.assemble(MAT, dev(pr.rho), None if mask is None else dev(mask)))
    Kref = O.assemble(elem, m.coords, m.cells, pr.rho, rp, ci, mask=mask)
    err = row_scaled_err(rp, K, Kref)
    print(f"elem={elem} skew={skew} mask={use_mask} K row-scaled err {err:.2e}")
    assert err <= TOL[api.FP64]


@pytest.mark.parametrize("elem,skew", [(e, None) for e in ELEMS] + [(I.QUAD4, "kink"), (I.HEX8, "kink")])
def test_assemble_fp32(elem, skew):
    pr, m, pat, rp, ci = _setup(elem, skew=skew)
    Kref = O.assemble(elem, m.coords, m.cells, pr.rho, rp, ci, mask=pr.mask)
    K32 = host(pat.assemble(MAT, dev(pr.rho, torch.float32), dev(pr.mask), prec=api.FP32))
    rho32 = pr.rho.astype(np.float32).astype(np.float64)
    Kref32 = O.assemble(elem, m.coords, m.cells, rho32, rp, ci, mask=pr.mask)
    e32 = row_scaled_err(rp, K32, Kref32)
    print(f"elem={elem} FP32 K err {e32:.2e} (vs FP64 oracle at the same densities)")
    assert e32 <= TOL[api.FP32]
    assert row_scaled_err(rp, host(pat.assemble(MAT, dev(pr.rho), dev(pr.mask))), Kref) <= 1e-12


@pytest.mark.parametrize("elem", ELEMS)
def test_bf16_form_refused(elem):
    """SOPTX_BF16_FP32ACC misses the 1e-5 bound, so every per-call entry point
    refuses it with SOPTX_E_INVALID_ARG before touching its outputs."""
    pr, m, pat, rp, ci = _setup(elem)
    rho32, u = dev(pr.rho, torch.float32), dev(pr.u)
    K = torch.full((pat.nnz,), 7.0, dtype=torch.float64, device="cuda")
    dc = torch.full((m.n_cells,), 7.0, dtype=torch.float32, device="cuda")
    c = torch.full((2,), 7.0, dtype=torch.float64, device="cuda")
    calls = [
        lambda: pat.assemble(MAT, rho32, dev(pr.mask), out=K, prec=api.BF16_FP32ACC),
        lambda: pat.sensitivity(MAT, rho32, u, out=dc, prec=api.BF16_FP32ACC),
        lambda: pat.compliance(MAT, rho32, u, out=c, prec=api.BF16_FP32ACC),
        lambda: pat.evaluate(MAT, rho32, u, dc=dc, c=c, prec=api.BF16_FP32ACC),
        lambda: pat.backward(MAT, rho32, K, out=dc, prec=api.BF16_FP32ACC),
    ]
    for call in calls:
        with pytest.raises(_lib.SoptxError) as ei:
            call()
        assert ei.value.code == -1
    torch.cuda.synchronize()
    assert bool((K == 7.0).all()) and bool((dc == 7.0).all()) and bool((c == 7.0).all())


@pytest.mark.parametrize("elem", ELEMS)
@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
def test_sensitivity_compliance(elem, prec):
    pr, m, pat, rp, ci = _setup(elem)
    tdt = torch.float64 if prec == api.FP64 else torch.float32
    rho = pr.rho if prec == api.FP64 else pr.rho.astype(np.float32).astype(np.float64)
    u = pr.u
    dc = host(pat.sensitivity(MAT, dev(rho, tdt), dev(u), prec=prec)).astype(np.float64)
    c = host(pat.compliance(MAT, dev(rho, tdt), dev(u), dev(pr.f), prec=prec))
    dc_ref = O.sensitivity(elem, m.coords, m.cells, rho, u)
    c_ref = O.compliance(elem, m.coords, m.cells, rho, u, pr.f)
    scale = abs_energy(m, u, np.arange(m.n_cells))
    cond_err = np.max(np.abs(dc - dc_ref) / (dE(rho) * scale))
    plain = np.max(np.abs(dc - dc_ref) / np.abs(dc_ref))
    c_err = abs(c[0] - c_ref[0]) / np.sum(E(rho) * scale)
    print(f"elem={elem} prec={prec} dc cond-scaled {cond_err:.2e} plain {plain:.2e} c {c_err:.2e}")
    assert cond_err <= TOL[prec]
    assert c_err <= TOL[prec]
    assert abs(c[1] - c_ref[1]) <= 1e-14 * np.sum(np.abs(pr.f * u))
    # fused entry point equals the separate calls bit for bit
    dc2, c2 = pat.evaluate(MAT, dev(rho, tdt), dev(u), dev(pr.f), prec=prec)
    assert np.array_equal(host(dc2).astype(np.float64), dc) and np.array_equal(host(c2), c)


@pytest.mark.parametrize("elem", [I.QUAD4, I.HEX8, I.TET10])
def test_sensitivity_on_solved_field(elem):
    """Solved fields are ill-conditioned for u^T K u; FP64 and FP32 (with the
    FP64 rigid-motion removal) stay within their bounds on the condition-scaled metric."""
    pr, m, pat, rp, ci = _setup(elem)
    f = np.zeros(m.ndof)
    free = np.nonzero(pr.mask == 0)[0]
    f[free[-1]] = -1.0
    K = O.assemble(elem, m.coords, m.cells, pr.rho, rp, ci, mask=pr.mask)
    u = O.solve(rp, ci, K, f)
    dc_ref = O.sensitivity(elem, m.coords, m.cells, pr.rho, u)
    scale = abs_energy(m, u, np.arange(m.n_cells))
    for prec, tdt in [(api.FP64, torch.float64), (api.FP32, torch.float32)]:
        rho = pr.rho if prec == api.FP64 else pr.rho.astype(np.float32).astype(np.float64)
        ref = dc_ref if prec == api.FP64 else O.sensitivity(elem, m.coords, m.cells, rho, u)
        dc = host(pat.sensitivity(MAT, dev(rho, tdt), dev(u), prec=prec)).astype(np.float64)
        cond_err = np.max(np.abs(dc - ref) / (dE(rho) * scale))
        plain = np.max(np.abs(dc - ref) / np.abs(ref))
        print(f"elem={elem} prec={prec} solved-field dc cond-scaled {cond_err:.2e} plain {plain:.2e}")
        assert cond_err <= TOL[prec]


@pytest.mark.parametrize("elem", ELEMS)
@pytest.mark.parametrize("use_mask", [False, True])
def test_backward(elem, use_mask):
    pr, m, pat, rp, ci = _setup(elem)
    rng = np.random.default_rng(11)
    Kbar = rng.standard_normal(ci.size)
    mask = pr.mask if use_mask else None
    dr = host(pat.backward(MAT, dev(pr.rho), dev(Kbar), None if mask is None else dev(mask)))
    Kb = Kbar.copy()
    if mask is not None:
        rows = np.repeat(np.arange(m.ndof), np.diff(rp))
        Kb[(mask[rows] != 0) | (mask[ci] != 0)] = 0.0
    ref = O.assemble_backward(elem, m.coords, m.cells, pr.rho, rp, ci, Kb)
    # scale: E' sum |Kbar| |K_e^0| over the element's slots
    scale = np.abs(ref) + 1e-300
    Kabs = O.assemble_backward(elem, m.coords, m.cells, pr.rho, rp, ci, np.abs(Kb))
    err = np.max(np.abs(dr - ref) / np.maximum(np.abs(Kabs), scale))
    print(f"elem={elem} mask={use_mask} backward err {err:.2e}")
    assert err <= 1e-12
    # Kbar = -u u^T reproduces the sensitivity (App. D)
    rows = np.repeat(np.arange(m.ndof), np.diff(rp))
    Kb2 = -pr.u[rows] * pr.u[ci]
    d2 = host(pat.backward(MAT, dev(pr.rho), dev(Kb2)))
    dc = host(pat.sensitivity(MAT, dev(pr.rho), dev(pr.u)))
    sc = dE(pr.rho) * abs_energy(m, pr.u, np.arange(m.n_cells))
    assert np.max(np.abs(d2 - dc) / sc) <= 1e-12


@pytest.mark.parametrize("elem", [I.QUAD4, I.HEX8])
def test_p4_and_plane_strain_and_noninteger_p(elem):
    pr, m, pat, rp, ci = _setup(elem)
    for mat in [api.Material(p=4.0), api.Material(p=2.5, nu=0.25, plane_strain=1), api.Material(E0=2.0, Emin=1e-6)]:
        K = host(pat.assemble(mat, dev(pr.rho)))
        Kref = O.assemble(elem, m.coords, m.cells, pr.rho, rp, ci, E0=mat.E0, Emin=mat.Emin, p=mat.p,
                          nu=mat.nu, plane_strain=mat.plane_strain)
        assert row_scaled_err(rp, K, Kref) <= 1e-12
        dc = host(pat.sensitivity(mat, dev(pr.rho), dev(pr.u)))
        ref = O.sensitivity(elem, m.coords, m.cells, pr.rho, pr.u, E0=mat.E0, Emin=mat.Emin, p=mat.p,
                            nu=mat.nu, plane_strain=mat.plane_strain)
        assert np.max(np.abs(dc - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("elem", ELEMS)
def test_determinism_and_streams(elem):
    pr, m, pat, rp, ci = _setup(elem)
    rho, mask, u = dev(pr.rho), dev(pr.mask), dev(pr.u)
    K1 = host(pat.assemble(MAT, rho, mask))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        Ka = pat.assemble(MAT, rho, mask, stream=s1)
        da, ca = pat.evaluate(MAT, rho, u, stream=s1)
    with torch.cuda.stream(s2):
        Kb = pat.assemble(MAT, rho, mask, stream=s2)
        db, cb = pat.evaluate(MAT, rho, u, stream=s2)
    torch.cuda.synchronize()
    assert np.array_equal(K1, host(Ka)) and np.array_equal(K1, host(Kb))
    assert np.array_equal(host(da), host(db)) and np.array_equal(host(ca), host(cb))


def test_edge_cases():
    # single element of each type
    for elem, mesh in [(I.QUAD4, I.quad_grid(1, 1)), (I.HEX8, I.hex_grid(1, 1, 1)),
                       (I.TRI3, I.tri_grid(1, 1)), (I.TET10, I.kuhn_p2_tets(1, 1, 1))]:
        m = mesh
        if elem in (I.TRI3, I.TET10):
            m = I.Mesh(elem, mesh.coords, mesh.cells[:1])
            used = np.unique(m.cells)
            remap = -np.ones(mesh.n_nodes, dtype=np.int64)
            remap[used] = np.arange(used.size)
            m = I.Mesh(elem, mesh.coords[used], remap[m.cells].astype(np.int32))
        pat = api.Pattern(elem, m.coords, m.cells)
        rho = np.array([0.5] * m.n_cells)
        K = host(pat.assemble(MAT, dev(rho)))
        rp, ci = O.pattern(elem, m.n_nodes, m.cells)
        Kref = O.assemble(elem, m.coords, m.cells, rho, rp, ci)
        assert row_scaled_err(rp, K, Kref) <= 1e-12
    # empty mesh: no cells, no nodes
    pat = api.Pattern(I.HEX8, np.zeros((0, 3)), np.zeros((0, 8), dtype=np.int32))
    assert pat.nnz == 0 and pat.ndof == 0
    rho = torch.zeros(0, dtype=torch.float64, device="cuda:0")
    pat.assemble(MAT, rho, out=torch.zeros(0, dtype=torch.float64, device="cuda:0"))
    c = pat.compliance(MAT, rho, torch.zeros(0, dtype=torch.float64, device="cuda:0"))
    assert host(c)[0] == 0.0
    # isolated node (no element): empty rows, rest unchanged
    m = I.quad_grid(2, 2)
    coords = np.vstack([m.coords, [[10.0, 10.0]]])
    pat = api.Pattern(I.QUAD4, coords, m.cells)
    rp, ci = O.pattern(I.QUAD4, coords.shape[0], m.cells)
    drp, dci = pat.pattern()
    assert np.array_equal(drp, rp) and np.array_equal(dci, ci)
    rho = np.linspace(0.1, 1, m.n_cells)
    assert row_scaled_err(rp, host(pat.assemble(MAT, dev(rho))), O.assemble(1, coords, m.cells, rho, rp, ci)) <= 1e-12


def test_argument_errors_raise():
    pr, m, pat, rp, ci = _setup(I.QUAD4)
    with pytest.raises(ValueError):
        pat.assemble(MAT, dev(pr.rho, torch.float32))  # wrong dtype for FP64
    with pytest.raises(ValueError):
        pat.assemble(MAT, dev(pr.rho[:-1]))
    with pytest.raises(Exception):
        pat.assemble(api.Material(nu=0.5), dev(pr.rho))


@pytest.mark.parametrize("elem", ELEMS)
def test_shuffled_numbering(elem):
    """Nodes and elements renumbered by a seeded permutation: a group's nodes
    are then no longer consecutive rows, and an element's nodes are far apart.
    K, dc and c against the oracle on the renumbered mesh."""
    pr = I.small_problem(elem, seed=61)
    m0 = pr.mesh
    rng = np.random.default_rng(62)
    pn = rng.permutation(m0.n_nodes)       # new id of old node i: pn[i]
    pe = rng.permutation(m0.n_cells)       # old element of new element k: pe[k]
    coords = np.empty_like(m0.coords)
    coords[pn] = m0.coords
    cells = pn[m0.cells[pe]].astype(np.int32)
    rho = pr.rho[pe]
    m = I.Mesh(elem, coords, cells)
    u = np.empty(m.ndof)
    u.reshape(-1, m.dim)[pn] = pr.u.reshape(-1, m.dim)
    pat = api.Pattern(elem, coords, cells)
    rp, ci = O.pattern(elem, m.n_nodes, cells)
    drp, dci = pat.pattern()
    assert np.array_equal(drp, rp) and np.array_equal(dci, ci)
    K = host(pat.assemble(MAT, dev(rho)))
    err = row_scaled_err(rp, K, O.assemble(elem, coords, cells, rho, rp, ci))
    dc, c = pat.evaluate(MAT, dev(rho), dev(u))
    dref = O.sensitivity(elem, coords, cells, rho, u)
    cref = O.compliance(elem, coords, cells, rho, u)
    sc = dE(rho) * abs_energy(m, u, np.arange(m.n_cells))
    derr = float(np.max(np.abs(host(dc) - dref) / sc))
    cerr = abs(float(host(c)[0]) - cref[0]) / float(np.sum(E(rho) * abs_energy(m, u, np.arange(m.n_cells))))
    print(f"elem={elem} shuffled: K {err:.2e} dc {derr:.2e} c {cerr:.2e}")
    assert err <= TOL[api.FP64] and derr <= TOL[api.FP64] and cerr <= TOL[api.FP64]


@pytest.mark.parametrize("elem", [I.QUAD4, I.HEX8, I.TET10])
def test_dirichlet_extreme_masks(elem):
    """Every dof fixed (K becomes the identity on the pattern) and only the
    last dof fixed (a ragged last chunk of the Dirichlet launch)."""
    pr, m, pat, rp, ci = _setup(elem)
    rows = np.repeat(np.arange(m.ndof), np.diff(rp))
    K = host(pat.assemble(MAT, dev(pr.rho), dev(np.ones(m.ndof, dtype=np.uint8))))
    assert np.array_equal(K, (rows == ci).astype(np.float64))
    last = np.zeros(m.ndof, dtype=np.uint8)
    last[-1] = 1
    K = host(pat.assemble(MAT, dev(pr.rho), dev(last)))
    Kref = O.assemble(elem, m.coords, m.cells, pr.rho, rp, ci, mask=last)
    touched = (rows == m.ndof - 1) | (ci == m.ndof - 1)
    assert np.array_equal(K[touched], Kref[touched])  # exact 0 / 1
    assert row_scaled_err(rp, K, Kref) <= TOL[api.FP64]
