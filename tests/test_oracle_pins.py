"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed
forms, exact symbolic integrals by an independent route (tests/exact_fe.py),
invariants (symmetry, rigid-body null space, linear patch test, compliance
identities), brute force on tiny inputs, finite differences, and the few
numbers the paper prints (tests/golden/).
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import exact_fe
from oracle import oracle as O
from paper_2505_02438_amd import api
from paper_2505_02438_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ELEMS = [I.QUAD4, I.TRI3, I.HEX8, I.TET10]

UNIT = {
    I.QUAD4: [(0, 0), (1, 0), (1, 1), (0, 1)],
    I.TRI3: [(0, 0), (1, 0), (0, 1)],
    I.HEX8: [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)],
}


def _f(p):
    return np.array([float(Fraction(c)) for c in p])


def _nodes(elem, d):
    """All node coordinates (floats) of the affine element whose map is defined
    by d (quad: d[0], d[1], d[3]; hex: d[0], d[1], d[3], d[4]; simplices: vertices)."""
    if elem == I.QUAD4:
        x0, a, b = _f(d[0]), _f(d[1]) - _f(d[0]), _f(d[3]) - _f(d[0])
        return np.array([x0, x0 + a, x0 + a + b, x0 + b])
    if elem == I.HEX8:
        x0 = _f(d[0])
        a, b, c = _f(d[1]) - x0, _f(d[3]) - x0, _f(d[4]) - x0
        return np.array([x0, x0 + a, x0 + a + b, x0 + b, x0 + c, x0 + a + c, x0 + a + b + c, x0 + b + c])
    if elem == I.TRI3:
        return np.array([_f(p) for p in d[:3]])
    vv = [_f(p) for p in d[:4]]
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    return np.array(vv + [0.5 * (vv[a] + vv[b]) for a, b in edges])


TET_UNIT = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]

# skewed affine elements with rational map-defining vertices
SKEW = {
    I.QUAD4: [("1/3", "1/5"), ("2", "1/2"), None, ("3/4", "7/4")],
    I.TRI3: [("1/3", "1/5"), ("2", "1/2"), ("3/4", "7/4")],
    I.HEX8: [("1/3", "1/5", "0"), ("2", "1/2", "1/7"), None, ("3/4", "7/4", "1/3"),
             ("1/2", "1/3", "9/5")],
    I.TET10: [("1/3", "1/5", "0"), ("2", "1/2", "1/7"), ("3/4", "7/4", "1/3"), ("1/2", "1/3", "9/5")],
}


def _defining(elem, shape):
    if shape == "skew":
        return SKEW[elem]
    return TET_UNIT if elem == I.TET10 else UNIT[elem]


# ------------------------------------------------------------ element matrices

def test_q1_quad_unit_square_closed_form():
    nu = 0.3
    ab = np.loadtxt(os.path.join(GOLDEN, "q1_quad_unit_square_row0.txt"))
    row0 = (ab[:, 0] + ab[:, 1] * nu) / (1 - nu * nu)
    Ke = O.element_ke0(I.QUAD4, np.array(UNIT[I.QUAD4], float), nu)
    np.testing.assert_allclose(Ke[0], row0, rtol=0, atol=1e-15)
    assert abs(np.trace(Ke) - 360 / 91) < 1e-14
    ev = np.sort(np.linalg.eigvalsh(Ke))
    np.testing.assert_allclose(ev[:3], 0, atol=1e-14)
    np.testing.assert_allclose(ev[3:], [45 / 91, 45 / 91, 70 / 91, 70 / 91, 130 / 91], rtol=1e-13)


def test_q1_hex_unit_cube_closed_form():
    Ke = O.element_ke0(I.HEX8, np.array(UNIT[I.HEX8], float), 0.3)
    # K[0,0] = (lambda + 4 mu)/9 with lambda = 15/26, mu = 5/13
    assert abs(Ke[0, 0] - 55 / 234) < 1e-15
    assert abs(np.trace(Ke) - 220 / 39) < 1e-13
    ev = np.sort(np.linalg.eigvalsh(Ke))
    assert np.all(np.abs(ev[:6]) < 1e-14) and ev[6] > 1e-2
    assert abs(ev[-1] - 1.25) < 1e-13


def test_p1_tri_unit_closed_form():
    Ke = O.element_ke0(I.TRI3, np.array(UNIT[I.TRI3], float), 0.3)
    assert abs(Ke[0, 0] - 135 / 182) < 1e-15
    assert abs(np.trace(Ke) - 270 / 91) < 1e-14


@pytest.mark.parametrize("elem", ELEMS)
@pytest.mark.parametrize("shape", ["unit", "skew"])
def test_ke_matches_exact_symbolic(elem, shape):
    """Standard-quadrature K_e^0 equals the exact integral of the Lame form."""
    d = _defining(elem, shape)
    ex = np.array(exact_fe.exact_ke0(elem, d), dtype=float)
    Ke = O.element_ke0(elem, _nodes(elem, d), 0.3)
    assert np.max(np.abs(Ke - ex)) <= 4e-15 * np.max(np.abs(ex))


@pytest.mark.parametrize("elem", ELEMS)
def test_plane_strain_and_nu_matches_exact(elem):
    d = _defining(elem, "skew")
    nu = Fraction(1, 4)
    for ps in ([0, 1] if I.ELEM_DIM[elem] == 2 else [0]):
        ex = np.array(exact_fe.exact_ke0(elem, d, nu=nu, plane_strain=bool(ps)), float)
        Ke = O.element_ke0(elem, _nodes(elem, d), float(nu), ps)
        assert np.max(np.abs(Ke - ex)) <= 4e-15 * np.max(np.abs(ex))


def _rigid_modes(coords, dim):
    n = coords.shape[0]
    modes = []
    for a in range(dim):
        r = np.zeros((n, dim))
        r[:, a] = 1.0
        modes.append(r.ravel())
    pairs = [(0, 1)] if dim == 2 else [(0, 1), (0, 2), (1, 2)]
    for a, b in pairs:
        r = np.zeros((n, dim))
        r[:, a] = -coords[:, b]
        r[:, b] = coords[:, a]
        modes.append(r.ravel())
    return modes


@pytest.mark.parametrize("elem", ELEMS)
def test_ke_symmetric_psd_rigid_nullspace(elem):
    prob = I.small_problem(elem, seed=11)
    m = prob.mesh
    for e in [0, m.n_cells // 2, m.n_cells - 1]:
        xe = m.coords[m.cells[e]]
        Ke = O.element_ke0(elem, xe, 0.3)
        nrm = np.abs(Ke).max()
        assert np.abs(Ke - Ke.T).max() <= 1e-15 * nrm
        for r in _rigid_modes(xe, m.dim):
            assert np.abs(Ke @ r).max() <= 1e-13 * nrm * np.abs(r).max()
        ev = np.linalg.eigvalsh(Ke)
        nz = 3 if m.dim == 2 else 6
        assert np.sum(np.abs(ev) < 1e-12 * nrm) == nz
        assert ev.min() > -1e-12 * nrm


# ------------------------------------------------------ quadrature, basis, D

@pytest.mark.parametrize("elem", ELEMS)
def test_quadrature_exact_for_design_degree(elem):
    """Each rule integrates every monomial of its design degree exactly."""
    from math import factorial
    pts, w = O.quadrature(elem)
    dim = I.ELEM_DIM[elem]
    simplex = elem in (I.TRI3, I.TET10)
    deg = {I.QUAD4: 3, I.HEX8: 3, I.TRI3: 1, I.TET10: 2}[elem]
    import itertools
    for mono in itertools.product(range(deg + 1), repeat=dim):
        if simplex and sum(mono) > deg:
            continue
        q = np.sum(w * np.prod(pts ** np.array(mono), axis=1))
        if simplex:
            ex = np.prod([factorial(a) for a in mono]) / factorial(sum(mono) + dim)
        else:
            ex = np.prod([1.0 / (a + 1) for a in mono])
        assert abs(q - ex) < 1e-15, (mono, q, ex)


@pytest.mark.parametrize("elem", ELEMS)
def test_basis_partition_of_unity_and_nodality(elem):
    nen = I.ELEM_NEN[elem]
    ref = {I.QUAD4: UNIT[I.QUAD4], I.HEX8: UNIT[I.HEX8], I.TRI3: UNIT[I.TRI3],
           I.TET10: _nodes(I.TET10, TET_UNIT)}[elem]
    for k, xi in enumerate(np.array(ref, float)):
        phi, dphi = O.ref_basis(elem, xi)
        np.testing.assert_allclose(phi, np.eye(nen)[k], atol=1e-15)
        np.testing.assert_allclose(dphi.sum(axis=0), 0, atol=1e-14)


def test_D_matrix_invariants():
    E, nu = 2.5, 0.3
    D3 = O.D_matrix(3, E, nu)
    # hydrostatic strain -> pressure with bulk term E/(1-2nu); shear modulus mu
    s = D3 @ np.array([1, 1, 1, 0, 0, 0.0])
    np.testing.assert_allclose(s[:3], E / (1 - 2 * nu), rtol=1e-15)
    assert abs(D3[3, 3] - E / (2 * (1 + nu))) < 1e-15
    # uniaxial stress: plane-stress D inverts to compliance [[1,-nu],[-nu,1]]/E
    D2 = O.D_matrix(2, E, nu)
    C = np.linalg.inv(D2[:2, :2])
    np.testing.assert_allclose(C, np.array([[1, -nu], [-nu, 1]]) / E, rtol=1e-14)
    assert abs(D2[2, 2] - E / (2 * (1 + nu))) < 1e-15
    # plane strain: D = the 3D matrix restricted to (xx, yy, xy)
    D2s = O.D_matrix(2, E, nu, plane_strain=1)
    np.testing.assert_allclose(D2s, D3[np.ix_([0, 1, 5], [0, 1, 5])], rtol=1e-15)


# ---------------------------------------------------------------- patterns

def _brute_pattern(elem, mesh):
    d = mesh.dim
    s = set()
    for cell in mesh.cells:
        dofs = [d * int(n) + a for n in cell for a in range(d)]
        for r in dofs:
            for c in dofs:
                s.add((r, c))
    s = sorted(s)
    row_ptr = np.zeros(mesh.ndof + 1, dtype=np.int64)
    for r, _ in s:
        row_ptr[r + 1] += 1
    return np.cumsum(row_ptr), np.array([c for _, c in s], dtype=np.int32)


@pytest.mark.parametrize("elem", ELEMS)
def test_pattern_bruteforce(elem):
    prob = I.small_problem(elem, seed=3)
    rp, ci = O.pattern(elem, prob.mesh.n_nodes, prob.mesh.cells)
    brp, bci = _brute_pattern(elem, prob.mesh)
    assert np.array_equal(rp, brp) and np.array_equal(ci, bci)


def test_pattern_bruteforce_shuffled_unstructured():
    """Arbitrary node numbering and element order: still the sorted unique set."""
    rng = np.random.default_rng(5)
    m = I.kuhn_p2_tets(2, 2, 1, jitter=0.1, rng=rng)
    perm = rng.permutation(m.n_nodes)
    cells = perm[m.cells][rng.permutation(m.n_cells)].astype(np.int32)
    coords = np.empty_like(m.coords)
    coords[perm] = m.coords
    mm = I.Mesh(m.elem, coords, cells)
    rp, ci = O.pattern(mm.elem, mm.n_nodes, mm.cells)
    brp, bci = _brute_pattern(mm.elem, mm)
    assert np.array_equal(rp, brp) and np.array_equal(ci, bci)


@pytest.mark.parametrize("nx,ny", [(1, 1), (4, 3), (60, 20)])
def test_pattern_nnz_closed_form_q1_2d(nx, ny):
    m = I.quad_grid(nx, ny)
    rp, ci = O.pattern(m.elem, m.n_nodes, m.cells)
    assert rp[-1] == 4 * (3 * nx + 1) * (3 * ny + 1)


@pytest.mark.parametrize("n", [(1, 1, 1), (3, 2, 4), (12, 4, 4)])
def test_pattern_nnz_closed_form_q1_3d(n):
    m = I.hex_grid(*n)
    rp, ci = O.pattern(m.elem, m.n_nodes, m.cells)
    assert rp[-1] == 9 * (3 * n[0] + 1) * (3 * n[1] + 1) * (3 * n[2] + 1)


@pytest.mark.parametrize("nx,ny", [(1, 1), (5, 3)])
def test_pattern_nnz_closed_form_tri(nx, ny):
    m = I.tri_grid(nx, ny)
    rp, ci = O.pattern(m.elem, m.n_nodes, m.cells)
    N = (nx + 1) * (ny + 1)
    E = nx * (ny + 1) + (nx + 1) * ny + nx * ny
    assert rp[-1] == 4 * (N + 2 * E)


def test_paper_dof_counts():
    with open(os.path.join(GOLDEN, "paper_values.json")) as fh:
        pv = json.load(fh)
    for key, dims in [("cantilever3d_60x20x4", (60, 20, 4)), ("cantilever3d_120x40x8", (120, 40, 8))]:
        m = I.hex_grid(*dims)
        assert m.ndof == pv[key]["dofs"]
        assert m.n_cells == pv[key]["densities"]


def test_kuhn_mesh_conforming_positive_affine():
    rng = np.random.default_rng(9)
    m = I.kuhn_p2_tets(3, 2, 2, jitter=0.15, rng=rng)
    X = m.coords[m.cells]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    assert np.all(np.linalg.det(J) > 0)
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    for k, (a, b) in enumerate(edges):
        np.testing.assert_allclose(X[:, 4 + k], 0.5 * (X[:, a] + X[:, b]), atol=1e-15)
    # every node used, each P2 node shared consistently (conforming): every
    # triangular face appears once (boundary) or twice (interior)
    assert np.unique(m.cells).size == m.n_nodes
    faces = {}
    for cell in m.cells:
        for f in [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]:
            key = tuple(sorted(int(cell[i]) for i in f))
            faces[key] = faces.get(key, 0) + 1
    assert set(faces.values()) <= {1, 2}
    nb = sum(1 for v in faces.values() if v == 1)
    assert nb == 2 * (2 * (3 * 2 + 3 * 2 + 2 * 2))  # 2 triangles per boundary square


def test_tri_mesh_positive():
    rng = np.random.default_rng(9)
    m = I.tri_grid(9, 7, jitter=0.2, rng=rng)
    X = m.coords[m.cells]
    det = (X[:, 1, 0] - X[:, 0, 0]) * (X[:, 2, 1] - X[:, 0, 1]) - (X[:, 1, 1] - X[:, 0, 1]) * (X[:, 2, 0] - X[:, 0, 0])
    assert np.all(det > 0)


# ------------------------------------------------------------ global invariants

def _assemble_all(prob, mask=None, p=None):
    m = prob.mesh
    rp, ci = O.pattern(m.elem, m.n_nodes, m.cells)
    K = O.assemble(m.elem, m.coords, m.cells, prob.rho, rp, ci, p=prob.p if p is None else p, mask=mask)
    return rp, ci, K


@pytest.mark.parametrize("elem", ELEMS)
def test_assembled_rigid_modes_and_symmetry(elem):
    prob = I.small_problem(elem, seed=21)
    m = prob.mesh
    rp, ci, K = _assemble_all(prob)
    rows = np.repeat(np.arange(m.ndof), np.diff(rp))
    A = np.zeros((m.ndof, m.ndof))
    A[rows, ci] = K
    nrm = np.abs(A).max()
    assert np.abs(A - A.T).max() <= 1e-15 * nrm
    for r in _rigid_modes(m.coords, m.dim):
        assert np.abs(O.spmv(rp, ci, K, r)).max() <= 1e-13 * nrm * np.abs(r).max()


def _voigt(eps, dim):
    if dim == 2:
        return np.array([eps[0, 0], eps[1, 1], 2 * eps[0, 1]])
    return np.array([eps[0, 0], eps[1, 1], eps[2, 2], 2 * eps[1, 2], 2 * eps[0, 2], 2 * eps[0, 1]])


def _volumes(mesh):
    X = mesh.coords[mesh.cells]
    if mesh.elem == I.QUAD4:
        a, b = X[:, 1] - X[:, 0], X[:, 3] - X[:, 0]
        return np.abs(a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0])
    if mesh.elem == I.TRI3:
        a, b = X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]
        return 0.5 * np.abs(a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0])
    if mesh.elem == I.HEX8:
        J = np.stack([X[:, 1] - X[:, 0], X[:, 3] - X[:, 0], X[:, 4] - X[:, 0]], axis=2)
        return np.abs(np.linalg.det(J))
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    return np.abs(np.linalg.det(J)) / 6.0


@pytest.mark.parametrize("elem", ELEMS)
def test_linear_patch_test(elem):
    """u = grad_u0 x gives s_e = |e| eps^T D eps exactly, dc and c in closed form,
    and (K u)_r = 0 at interior dofs for uniform density."""
    prob = I.small_problem(elem, seed=4)
    m = prob.mesh
    rng = np.random.default_rng(1)
    Gu = rng.standard_normal((m.dim, m.dim))
    u = (m.coords @ Gu.T).ravel()
    eps = 0.5 * (Gu + Gu.T)
    D = O.D_matrix(m.dim, 1.0, 0.3)
    ev = _voigt(eps, m.dim)
    e_dens = ev @ D @ ev
    vol = _volumes(m)
    s = O.element_energy(elem, m.coords, m.cells, u)
    np.testing.assert_allclose(s, vol * e_dens, rtol=1e-12)
    dc = O.sensitivity(elem, m.coords, m.cells, prob.rho, u)
    dE = 3 * prob.rho ** 2 * (1 - 1e-9)
    np.testing.assert_allclose(dc, -dE * vol * e_dens, rtol=1e-12)
    c = O.compliance(elem, m.coords, m.cells, prob.rho, u)
    E = 1e-9 + prob.rho ** 3 * (1 - 1e-9)
    assert abs(c[0] - np.sum(E * vol) * e_dens) <= 1e-12 * abs(c[0])
    # interior equilibrium for uniform density
    rho1 = np.full(m.n_cells, 0.7)
    rp, ci = O.pattern(elem, m.n_nodes, m.cells)
    K = O.assemble(elem, m.coords, m.cells, rho1, rp, ci)
    Ku = O.spmv(rp, ci, K, u)
    x = m.coords
    lo, hi = x.min(axis=0), x.max(axis=0)
    interior = np.all((x > lo + 1e-9) & (x < hi - 1e-9), axis=1)
    idx = (m.dim * np.nonzero(interior)[0][:, None] + np.arange(m.dim)).ravel()
    assert idx.size > 0
    assert np.abs(Ku[idx]).max() <= 1e-12 * np.abs(K).max() * np.abs(u).max()


def test_simp_law():
    m = I.quad_grid(2, 1)
    u = np.random.default_rng(2).standard_normal(m.ndof)
    s = O.element_energy(m.elem, m.coords, m.cells, u)
    for rho, p in [(0.0, 3.0), (1.0, 3.0), (0.5, 3.0), (0.37, 4.0)]:
        r = np.full(m.n_cells, rho)
        c = O.compliance(m.elem, m.coords, m.cells, r, u, p=p)
        E = 1e-9 + rho ** p * (1 - 1e-9)
        assert abs(c[0] - E * s.sum()) <= 1e-15 * abs(c[0]) + 1e-30
    # E(0) = Emin, E(1) = E0: compliance scales accordingly
    c0 = O.compliance(m.elem, m.coords, m.cells, np.zeros(m.n_cells), u)[0]
    c1 = O.compliance(m.elem, m.coords, m.cells, np.ones(m.n_cells), u)[0]
    assert abs(c0 / c1 - 1e-9) < 1e-20


def test_dirichlet_rows_cols():
    prob = I.small_problem(I.QUAD4, seed=8)
    m = prob.mesh
    rp, ci, K = _assemble_all(prob, mask=prob.mask)
    rows = np.repeat(np.arange(m.ndof), np.diff(rp))
    fixed = prob.mask.astype(bool)
    sel = fixed[rows] | fixed[ci]
    assert np.all(K[sel & (rows == ci)] == 1.0)
    assert np.all(K[sel & (rows != ci)] == 0.0)
    _, _, K0 = _assemble_all(prob)
    assert np.array_equal(K[~sel], K0[~sel])


# ------------------------------------------------------ compliance and sensitivity

def _solve_problem(prob):
    m = prob.mesh
    rp, ci, K = _assemble_all(prob, mask=prob.mask)
    f = prob.f.copy()
    f[prob.mask != 0] = 0.0
    u = O.solve(rp, ci, K, f)
    return rp, ci, K, f, u


@pytest.mark.parametrize("elem", ELEMS)
def test_compliance_identities_on_solved_field(elem):
    """f^T u = u^T K u = sum_e E_e s_e (Eq. cmpd; c is twice the strain energy)."""
    prob = I.small_problem(elem, seed=13)
    prob.f[:] = 0.0
    # a load on a free dof: the highest-numbered dof that is not fixed
    free = np.nonzero(prob.mask == 0)[0]
    prob.f[free[-1]] = -1.0
    prob.f[free[len(free) // 2]] = 0.5
    rp, ci, K, f, u = _solve_problem(prob)
    m = prob.mesh
    r = O.spmv(rp, ci, K, u) - f
    assert np.abs(r).max() <= 1e-10 * np.abs(f).max()
    uKu = u @ O.spmv(rp, ci, K, u)
    c = O.compliance(elem, m.coords, m.cells, prob.rho, u, f)
    assert abs(c[1] - uKu) <= 1e-9 * abs(uKu)
    assert abs(c[0] - uKu) <= 1e-9 * abs(uKu)


def test_fd_sensitivity_through_solve():
    """dc_e from the adjoint formula equals the central difference of c(rho) = f^T u(rho)."""
    prob = I.mbb_q1(6, 3, seed=1001)
    m = prob.mesh
    rp, ci, K, f, u = _solve_problem(prob)
    dc = O.sensitivity(m.elem, m.coords, m.cells, prob.rho, u)
    fd = np.zeros(m.n_cells)
    for e in range(m.n_cells):
        h = 1e-4 * prob.rho[e]
        vals = []
        for sgn in (+1, -1):
            r2 = prob.rho.copy()
            r2[e] += sgn * h
            K2 = O.assemble(m.elem, m.coords, m.cells, r2, rp, ci, mask=prob.mask)
            vals.append(f @ O.solve(rp, ci, K2, f))
        fd[e] = (vals[0] - vals[1]) / (2 * h)
    assert np.abs(fd - dc).max() <= 1e-6 * np.abs(dc).max()
    assert np.all(dc < 0)


@pytest.mark.parametrize("elem", [I.QUAD4, I.HEX8, I.TET10])
def test_backward_fd_and_adjoint_identity(elem):
    prob = I.small_problem(elem, seed=17)
    m = prob.mesh
    rp, ci = O.pattern(elem, m.n_nodes, m.cells)
    rng = np.random.default_rng(3)
    Kbar = rng.standard_normal(ci.size)
    dr = O.assemble_backward(elem, m.coords, m.cells, prob.rho, rp, ci, Kbar)
    # L(rho) = <Kbar, K(rho)> is a cubic in each rho_e: a central difference with
    # Richardson extrapolation over h and 2h is exact up to rounding
    for e in [0, m.n_cells // 3, m.n_cells - 1]:
        def L(x):
            r2 = prob.rho.copy()
            r2[e] = x
            return Kbar @ O.assemble(elem, m.coords, m.cells, r2, rp, ci)
        h = 0.05 * prob.rho[e]
        d1 = (L(prob.rho[e] + h) - L(prob.rho[e] - h)) / (2 * h)
        d2 = (L(prob.rho[e] + 2 * h) - L(prob.rho[e] - 2 * h)) / (4 * h)
        fd = (4 * d1 - d2) / 3
        assert abs(fd - dr[e]) <= 1e-9 * (abs(dr[e]) + np.abs(Kbar).max())
    # Kbar = -u u^T on the pattern reproduces the sensitivity dc
    u = prob.u
    rows = np.repeat(np.arange(m.ndof), np.diff(rp))
    Kbar2 = -u[rows] * u[ci]
    dr2 = O.assemble_backward(elem, m.coords, m.cells, prob.rho, rp, ci, Kbar2)
    dc = O.sensitivity(elem, m.coords, m.cells, prob.rho, u)
    np.testing.assert_allclose(dr2, dc, rtol=1e-11, atol=1e-14 * np.abs(dc).max())


@pytest.mark.slow
def test_paper_cantilever_initial_compliance():
    """Sec. 4.2: the 160x100 cantilever starts at compliance approximately 500
    (uniform density 0.4).  Also c(0.4)/c(1) = E(1)/E(0.4) for uniform density."""
    with open(os.path.join(GOLDEN, "paper_values.json")) as fh:
        ref = json.load(fh)["cantilever_160x100_initial_compliance"]["value"]
    m = I.quad_grid(160, 100)
    mask, f = I.cantilever2d_bc(m, load="bottom_right")
    rp, ci = O.pattern(m.elem, m.n_nodes, m.cells)
    cs = {}
    for rho0 in (0.4, 1.0):
        rho = np.full(m.n_cells, rho0)
        K = O.assemble(m.elem, m.coords, m.cells, rho, rp, ci, mask=mask)
        u = O.solve(rp, ci, K, f)
        c = O.compliance(m.elem, m.coords, m.cells, rho, u, f)
        assert abs(c[0] - c[1]) <= 1e-8 * c[1]
        cs[rho0] = c[1]
    assert abs(cs[0.4] - ref) <= 0.05 * ref
    E04 = 1e-9 + 0.4 ** 3 * (1 - 1e-9)
    assert abs(cs[0.4] / cs[1.0] - 1.0 / E04) <= 1e-8 / E04


@pytest.mark.parametrize("elem", [I.QUAD4, I.HEX8])
def test_nonaffine_q1_oracle(elem):
    """General (non-affine) Q1 elements, where K_e^0 is integrated with J at
    every Gauss point: symmetric, rigid modes in the null space, and the
    linear patch test: u_e^T K_e^0 u_e = |e| eps^T D eps for a linear field
    (quads: |e| by the shoelace formula; hexahedra: the energies add up to
    the box volume, the cells tiling it), and K u = 0 at interior dofs."""
    rng = np.random.default_rng(31)
    m0 = I.quad_grid(5, 4) if elem == I.QUAD4 else I.hex_grid(4, 3, 3)
    m = I.jitter_interior(m0, 0.3, rng)
    assert api.validate_mesh(m.elem, m.coords, m.cells) == -5          # not affine
    Gu = rng.standard_normal((m.dim, m.dim))
    u = (m.coords @ Gu.T).ravel()
    eps = 0.5 * (Gu + Gu.T)
    ev = _voigt(eps, m.dim)
    e_dens = ev @ O.D_matrix(m.dim, 1.0, 0.3) @ ev
    s = []
    for e in range(m.n_cells):
        Ke = O.element_ke0(elem, m.coords[m.cells[e]])
        assert np.abs(Ke - Ke.T).max() <= 1e-14 * np.abs(Ke).max()
        ue = u.reshape(-1, m.dim)[m.cells[e]].ravel()
        s.append(ue @ Ke @ ue)
    s = np.array(s)
    if elem == I.QUAD4:
        X = m.coords[m.cells]
        area = 0.5 * np.abs(sum(X[:, k, 0] * X[:, (k + 1) % 4, 1] - X[:, (k + 1) % 4, 0] * X[:, k, 1]
                                for k in range(4)))
        np.testing.assert_allclose(s, area * e_dens, rtol=1e-12)
    else:
        assert abs(s.sum() - 4 * 3 * 3 * e_dens) <= 1e-12 * abs(s.sum())
    rho1 = np.full(m.n_cells, 0.7)
    rp, ci = O.pattern(elem, m.n_nodes, m.cells)
    K = O.assemble(elem, m.coords, m.cells, rho1, rp, ci)
    Ku = O.spmv(rp, ci, K, u)
    x = m.coords
    lo, hi = x.min(axis=0), x.max(axis=0)
    interior = np.all((x > lo + 1e-9) & (x < hi - 1e-9), axis=1)
    idx = (m.dim * np.nonzero(interior)[0][:, None] + np.arange(m.dim)).ravel()
    assert idx.size > 0
    assert np.abs(Ku[idx]).max() <= 1e-12 * np.abs(K).max() * np.abs(u).max()
    for r in _rigid_modes(m.coords, m.dim):
        assert np.abs(O.spmv(rp, ci, K, r)).max() <= 1e-13 * np.abs(K).max() * np.abs(r).max()
    # the element energy (Gauss-point form) passes the same patch test
    se = O.element_energy(elem, m.coords, m.cells, u)
    if elem == I.QUAD4:
        np.testing.assert_allclose(se, area * e_dens, rtol=1e-12)
    else:
        np.testing.assert_allclose(se, s, rtol=1e-12)
