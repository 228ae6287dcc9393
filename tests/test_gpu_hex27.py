"""Q2 hexahedra (27-node triquadratic elements) on the GPU, through the C ABI:
the assembly with the Jacobian at every Gauss point (soptx_assemble_general:
one element per block, then the ascending-element gather) and the element
energies (soptx_evaluate_general) against the oracle, on straight and curved
(jittered) meshes; the full curved 60 x 20 x 20 cantilever on sampled rows
and elements, and c = u^T K u; optimisation iterations against the oracles.

Tolerances: K and dc by the row- and condition-scaled metrics of the Q1
tests (<= 1e-12); the sums c and f^T u relative to their absolute sums."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2505_02438_amd import _lib, api
from paper_2505_02438_amd import inputs as I

from gpu_util import dev, host

pytestmark = pytest.mark.gpu

H27 = I.HEX27


def _row_scaled(rp, Kg, Kr, rows=None):
    n = len(rp) - 1
    rix = np.repeat(np.arange(n), np.diff(rp))
    den = np.zeros(n)
    np.maximum.at(den, rix, np.abs(Kr))
    num = np.zeros(n)
    np.maximum.at(num, rix, np.abs(Kg - Kr))
    r = num / np.where(den > 0, den, 1.0)
    return float(np.max(r if rows is None else r[rows]))


def _mesh(dims, jitter, seed):
    rng = np.random.default_rng(seed)
    m = I.hex27_grid(*dims)
    return (I.jitter_interior(m, jitter, rng) if jitter else m), rng


@pytest.mark.parametrize("dims,jitter", [((1, 1, 1), 0.0), ((3, 2, 2), 0.0), ((3, 2, 2), 0.12), ((5, 3, 2), 0.1)])
def test_hex27_assembly_matches_oracle(dims, jitter):
    m, rng = _mesh(dims, jitter, 71)
    pat = api.Pattern.from_mesh(m, general=True)
    rho = rng.uniform(1e-3, 1.0, m.n_cells)
    mat = api.Material(E0=1.0, Emin=1e-9, nu=0.3, p=3.0)
    rp, ci = O.pattern(H27, m.n_nodes, m.cells)
    r2, c2 = pat.pattern()
    assert np.array_equal(r2, rp) and np.array_equal(c2, ci)
    mask = (rng.uniform(size=m.ndof) < 0.1).astype(np.uint8)
    for msk in (None, mask):
        K = host(pat.assemble_general(mat, dev(rho), None if msk is None else dev(msk)))
        Kr = O.assemble(H27, m.coords, m.cells, rho, rp, ci, mask=msk)
        err = _row_scaled(rp, K, Kr)
        print(f"Q2 hex {dims} jitter {jitter} mask={msk is not None}: row-scaled {err:.1e}")
        assert err <= 1e-12
        if msk is not None:
            fixed = np.nonzero(msk)[0]
            rows = np.repeat(np.arange(m.ndof), np.diff(rp))
            sel = np.isin(rows, fixed) | np.isin(ci, fixed)
            assert np.array_equal(K[sel], Kr[sel])
    # deterministic, and the affine-only calls refuse the handle
    assert torch.equal(pat.assemble_general(mat, dev(rho)), pat.assemble_general(mat, dev(rho)))
    with pytest.raises(_lib.SoptxError) as e:
        pat.assemble(mat, dev(rho))
    assert e.value.code == -2


def _scaled_dc(m, rho, u, dc_gpu, dc_ref, cells_idx, p=3.0):
    dE = p * rho ** (p - 1) * (1.0 - 1e-9)
    out = 0.0
    uu = u.reshape(-1, 3)
    for k, e in enumerate(cells_idx):
        Ke = O.element_ke0(H27, m.coords[m.cells[e]])
        ue = np.abs(uu[m.cells[e]].ravel())
        out = max(out, abs(dc_gpu[k] - dc_ref[k]) / (dE[e] * (ue @ np.abs(Ke) @ ue)))
    return out


@pytest.mark.parametrize("dims,jitter", [((3, 2, 2), 0.0), ((5, 3, 2), 0.12), ((4, 4, 3), 0.1)])
def test_hex27_evaluate_matches_oracle(dims, jitter):
    m, rng = _mesh(dims, jitter, 72)
    pat = api.Pattern.from_mesh(m, general=True)
    rho = rng.uniform(1e-3, 1.0, m.n_cells)
    u = rng.standard_normal(m.ndof)
    f = rng.standard_normal(m.ndof)
    mat = api.Material(E0=1.0, Emin=1e-9, nu=0.3, p=3.0)
    dc, c = pat.evaluate_general(mat, dev(rho), dev(u), f=dev(f))
    dc, c = host(dc), host(c)
    dref = O.sensitivity(H27, m.coords, m.cells, rho, u)
    cref = O.compliance(H27, m.coords, m.cells, rho, u, f)
    err = _scaled_dc(m, rho, u, dc, dref, range(m.n_cells))
    E = 1e-9 + rho ** 3 * (1 - 1e-9)
    cscale = float(np.sum(E * np.abs(dref) / (3 * rho ** 2 * (1 - 1e-9))))
    print(f"Q2 hex {dims}: dc scaled {err:.1e}, c {abs(c[0] - cref[0]) / cscale:.1e}")
    assert err <= 1e-12 and abs(c[0] - cref[0]) <= 1e-12 * cscale
    assert abs(c[1] - cref[1]) <= 1e-13 * float(np.abs(f) @ np.abs(u))
    # dc alone, and c alone without f
    dc2, _ = pat.evaluate_general(mat, dev(rho), dev(u))
    assert np.array_equal(host(dc2), dc)


def test_hex27_full_cantilever_sampled():
    """The 60 x 20 x 20 curved Q2 cantilever (the 120 x 40 x 40 box, the Q1
    cantilever's node lattice): K rows of sampled nodes against the oracle's
    assembly of their elements, sampled dc against the oracle, and
    c = sum_e E(rho_e) s_e against u^T K u from the assembled matrix."""
    pr = I.cantilever_hex27()
    m = pr.mesh
    pat = api.Pattern.from_mesh(m, general=True)
    mat = api.Material(E0=pr.E0, Emin=pr.Emin, nu=pr.nu, p=pr.p)
    rho_d = dev(pr.rho)
    K = pat.assemble_general(mat, rho_d, dev(pr.mask))
    rp, ci = pat.pattern()
    rng = np.random.default_rng(73)
    nodes = rng.choice(m.n_nodes, 40, replace=False)
    cells = np.nonzero(np.isin(m.cells, nodes).any(axis=1))[0]
    sub = m.cells[cells]
    rps, cis = O.pattern(H27, m.n_nodes, sub)
    Ks = O.assemble(H27, m.coords, sub, pr.rho[cells], rps, cis, mask=pr.mask)
    Kh = host(K)
    worst = 0.0
    for n in nodes:
        for a in range(3):
            r = 3 * n + a
            assert np.array_equal(ci[rp[r]:rp[r + 1]], cis[rps[r]:rps[r + 1]])
            kg, kr = Kh[rp[r]:rp[r + 1]], Ks[rps[r]:rps[r + 1]]
            worst = max(worst, float(np.max(np.abs(kg - kr)) / np.max(np.abs(kr))))
    print(f"full Q2 cantilever: {len(nodes)} sampled nodes ({len(cells)} elements), row-scaled {worst:.1e}")
    assert worst <= 1e-12
    u_d = dev(pr.u)
    dc, c = pat.evaluate_general(mat, rho_d, u_d, f=dev(pr.f))
    els = rng.choice(m.n_cells, 30, replace=False)
    dref = O.sensitivity(H27, m.coords, m.cells[els], pr.rho[els], pr.u)
    err = _scaled_dc(m, pr.rho, pr.u, host(dc)[els], dref, els)
    print(f"sampled dc scaled {err:.1e}")
    assert err <= 1e-12
    # c = u^T K(rho) u with no Dirichlet rows (u is zero on the fixed dofs)
    K0 = pat.assemble_general(mat, rho_d)
    uKu = float(torch.dot(u_d, pat.spmv(K0, u_d)))
    c0 = float(host(c)[0])
    print(f"c {c0!r}, u^T K u {uKu!r}")
    assert abs(c0 - uKu) <= 1e-11 * abs(uKu)
    assert abs(float(host(c)[1]) - float(pr.f @ pr.u)) <= 1e-12 * float(np.abs(pr.f) @ np.abs(pr.u))


def test_hex27_optimisation_iterations_match_oracle():
    """Three iterations of Algorithm 1 on a curved 8 x 2 x 2 Q2 cantilever
    (volume fraction 0.3, sensitivity filter r = 1.5, m = 0.2, eta = 0.5),
    all on the GPU, against the same iterations of the oracles."""
    from oracle import filters as OF
    from oracle import oc as OC
    from paper_2505_02438_amd import loop
    m = I.jitter_interior(I.hex27_grid(8, 2, 2), 0.1, np.random.default_rng(74))
    mask, f = I.clamp_x0_bc(m)
    res = loop.run(m, mask, f, 0.3, 1.5, max_iter=3, tol=0.0, cg_rtol=1e-12, general=True)
    rp, ci = O.pattern(H27, m.n_nodes, m.cells)
    H = OF.filter_matrix(OF.centroids(H27, m.coords, m.cells), 1.5)
    v = OF.volumes(H27, m.coords, m.cells)
    rho = np.full(m.n_cells, 0.3)
    for it in range(3):
        K = O.assemble(H27, m.coords, m.cells, rho, rp, ci, mask=mask)
        uo = O.solve(rp, ci, K, f)
        co = O.compliance(H27, m.coords, m.cells, rho, uo, f)[1]
        dco = O.sensitivity(H27, m.coords, m.cells, rho, uo)
        rho, *_ = OC.oc_update(rho, OF.sensitivity_filter(H, rho, dco), v, 0.3 * v.sum(), move=0.2, eta=0.5)
        print(f"iteration {it}: c {res.compliance[it]:.10f} / {co:.10f}")
        assert abs(res.compliance[it] - co) <= 1e-8 * co
    assert float(np.max(np.abs(host(res.rho) - rho))) <= 1e-6


def test_hex27_degenerate_meshes():
    """No cells and no nodes; nodes but no cells (c = [0, f^T u]); one element
    beside an isolated node (its rows empty, the rest as the oracle)."""
    mat = api.Material()
    pat = api.Pattern(H27, np.zeros((0, 3)), np.zeros((0, 27), dtype=np.int32), general=True)
    assert pat.nnz == 0 and pat.ndof == 0
    z = torch.zeros(0, dtype=torch.float64, device="cuda:0")
    pat.assemble_general(mat, z, out=torch.zeros(0, dtype=torch.float64, device="cuda:0"))
    _, c = pat.evaluate_general(mat, z, z, f=z)
    assert np.array_equal(host(c), [0.0, 0.0])
    x = np.random.default_rng(75).standard_normal((5, 3))
    pat = api.Pattern(H27, x, np.zeros((0, 27), dtype=np.int32), general=True)
    assert pat.nnz == 0 and pat.ndof == 15
    u, f = np.arange(15.0), np.linspace(-1, 1, 15)
    _, c = pat.evaluate_general(mat, z, dev(u), f=dev(f))
    assert host(c)[0] == 0.0 and abs(host(c)[1] - f @ u) <= 1e-13 * np.abs(f) @ np.abs(u)
    m = I.hex27_grid(1, 1, 1)
    coords = np.vstack([m.coords, [[5.0, 5.0, 5.0]]])
    pat = api.Pattern(H27, coords, m.cells, general=True)
    rp, ci = O.pattern(H27, coords.shape[0], m.cells)
    drp, dci = pat.pattern()
    assert np.array_equal(drp, rp) and np.array_equal(dci, ci) and rp[-1] == rp[-4]
    rho = np.array([0.4])
    K = host(pat.assemble_general(mat, dev(rho)))
    assert _row_scaled(rp, K, O.assemble(H27, coords, m.cells, rho, rp, ci)) <= 1e-12


def test_hex27_filter_stencil_and_oracle():
    """A straight Q2 grid: centroids (corner means) on a regular lattice, so
    the filter takes its stencil form; stencil and CSR forms bitwise equal,
    and the sensitivity filter bitwise equal to the oracle's."""
    from oracle import filters as OF
    m = I.hex27_grid(9, 5, 4)
    fs = api.Filter.from_mesh(m, 1.5)
    fc = api.Filter(m.elem, m.coords, m.cells, 1.5, csr_only=True)
    assert fs.stencil_size == 19 and fc.stencil_size == 0
    rng = np.random.default_rng(76)
    rho = rng.uniform(0.0, 1.0, m.n_cells)
    dc = -rng.exponential(1.0, m.n_cells)
    a, b = fs.sensitivity(dev(rho), dev(dc)), fc.sensitivity(dev(rho), dev(dc))
    assert torch.equal(a, b)
    H = OF.filter_matrix(OF.centroids(H27, m.coords, m.cells), 1.5)
    assert np.array_equal(host(a), OF.sensitivity_filter(H, rho, dc))
    v = OF.volumes(H27, m.coords, m.cells)
    np.testing.assert_allclose(host(fs.density(dev(rho))), OF.density_filter(H, v, rho), rtol=1e-14, atol=0)


@pytest.mark.parametrize("elem", [I.HEX8, H27])
def test_general_noninteger_exponent(elem):
    """p = 2.5 takes the pow branch of the SIMP law in the element kernels
    (assembly and energies) of both general element families."""
    rng = np.random.default_rng(77)
    m = I.jitter_interior(I.hex_grid(4, 3, 3) if elem == I.HEX8 else I.hex27_grid(3, 2, 2),
                          0.25 if elem == I.HEX8 else 0.1, rng)
    pat = api.Pattern.from_mesh(m, general=True)
    mat = api.Material(E0=2.0, Emin=1e-6, nu=0.25, p=2.5)
    rho = rng.uniform(0.01, 1.0, m.n_cells)
    u = rng.standard_normal(m.ndof)
    rp, ci = O.pattern(elem, m.n_nodes, m.cells)
    K = host(pat.assemble_general(mat, dev(rho)))
    Kr = O.assemble(elem, m.coords, m.cells, rho, rp, ci, E0=2.0, Emin=1e-6, p=2.5, nu=0.25)
    assert _row_scaled(rp, K, Kr) <= 1e-12
    dc, c = pat.evaluate_general(mat, dev(rho), dev(u))
    dref = O.sensitivity(elem, m.coords, m.cells, rho, u, E0=2.0, Emin=1e-6, p=2.5, nu=0.25)
    cref = O.compliance(elem, m.coords, m.cells, rho, u, None, E0=2.0, Emin=1e-6, p=2.5, nu=0.25)
    np.testing.assert_allclose(host(dc), dref, rtol=1e-12, atol=1e-12 * np.abs(dref).max())
    assert abs(host(c)[0] - cref[0]) <= 1e-12 * abs(cref[0])


def test_hex27_density_filter_iterations_match_oracle():
    """Three iterations with the density filter (Sec. 2.4) on a curved
    6 x 2 x 2 Q2 cantilever: the physical density F(rho) is assembled and
    evaluated, dc and dv go back through the filter's chain rule; against the
    same iterations of the oracles."""
    from oracle import filters as OF
    from oracle import oc as OC
    from paper_2505_02438_amd import loop
    m = I.jitter_interior(I.hex27_grid(6, 2, 2), 0.1, np.random.default_rng(78))
    mask, f = I.clamp_x0_bc(m)
    res = loop.run(m, mask, f, 0.4, 1.6, filt="density", max_iter=3, tol=0.0, cg_rtol=1e-12, general=True)
    rp, ci = O.pattern(H27, m.n_nodes, m.cells)
    H = OF.filter_matrix(OF.centroids(H27, m.coords, m.cells), 1.6)
    v = OF.volumes(H27, m.coords, m.cells)
    dv = OF.density_filter_backward(H, v, v)
    rho = np.full(m.n_cells, 0.4)
    for it in range(3):
        rt = OF.density_filter(H, v, rho)
        K = O.assemble(H27, m.coords, m.cells, rt, rp, ci, mask=mask)
        uo = O.solve(rp, ci, K, f)
        co = O.compliance(H27, m.coords, m.cells, rt, uo, f)[1]
        dco = O.sensitivity(H27, m.coords, m.cells, rt, uo)
        rho, *_ = OC.oc_update(rho, OF.density_filter_backward(H, v, dco), dv, 0.4 * v.sum(), move=0.2, eta=0.5)
        print(f"density filter, iteration {it}: c {res.compliance[it]:.10f} / {co:.10f}")
        assert abs(res.compliance[it] - co) <= 1e-8 * co
    assert float(np.max(np.abs(host(res.rho) - rho))) <= 1e-6
