"""Host side of the assembly with per-quadrature-point geometry: general Q1
meshes are accepted by the general build only, inverted cells are rejected,
and the contribution table lists, for every DIM x DIM block of K, exactly the
elements holding both nodes, in ascending element order, with the nodes'
local indices.  No GPU."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2505_02438_amd import _lib, api
from paper_2505_02438_amd import inputs as I


@pytest.mark.parametrize("elem", [I.QUAD4, I.HEX8, I.HEX27])
def test_contribution_table(elem):
    rng = np.random.default_rng(3)
    m0 = {I.QUAD4: lambda: I.quad_grid(6, 5), I.HEX8: lambda: I.hex_grid(4, 3, 3),
          I.HEX27: lambda: I.hex27_grid(2, 2, 1)}[elem]()
    m = I.jitter_interior(m0, 0.12 if elem == I.HEX27 else 0.3, rng)
    with pytest.raises(_lib.SoptxError) as e:
        api.host_plan(m.elem, m.coords, m.cells)
    # Q2 hexahedra are refused by the affine-only build even when straight
    assert e.value.code == (-2 if elem == I.HEX27 else -5)
    hp = api.host_plan(m.elem, m.coords, m.cells, general=True)
    rp, ci = O.pattern(elem, m.n_nodes, m.cells)
    np.testing.assert_array_equal(hp["row_ptr"], rp)
    np.testing.assert_array_equal(hp["col_idx"], ci)
    d, nen = m.dim, m.cells.shape[1]
    nblk = len(ci) // (d * d)
    gptr, gent, gnode = hp["gptr"], hp["gent"], hp["gnode"]
    assert len(gptr) == nblk + 1 and len(gent) == m.n_cells * nen * nen and gptr[-1] == len(gent)
    cells = m.cells
    for b in range(nblk):
        n = gnode[b]
        q = b - rp[d * n] // (d * d)
        J = ci[rp[d * n] + d * q] // d                    # the neighbour of block b
        got = [(g // (nen * nen), (g // nen) % nen, g % nen) for g in gent[gptr[b]:gptr[b + 1]]]
        want = [(e, int(np.nonzero(cells[e] == n)[0][0]), int(np.nonzero(cells[e] == J)[0][0]))
                for e in range(m.n_cells) if n in cells[e] and J in cells[e]]
        assert got == want, b


def test_inverted_cell_rejected():
    m = I.quad_grid(3, 3)
    c = m.coords.copy()
    # push an interior node past its neighbours: a cell turns inside out
    k = 1 * 4 + 1
    c[k] = [2.6, 2.6]
    with pytest.raises(_lib.SoptxError) as e:
        api.host_plan(m.elem, c, m.cells, general=True)
    assert e.value.code == -4
    # simplices stay affine-only: a curved P2 tetrahedron is refused
    pr = I.small_problem(I.TET10, seed=2)
    x = pr.mesh.coords.copy()
    x[pr.mesh.cells[0, 4]] += 0.05                       # an edge midpoint off its edge
    with pytest.raises(_lib.SoptxError) as e:
        api.host_plan(I.TET10, x, pr.mesh.cells, general=True)
    assert e.value.code == -5


def test_hex27_host_checks():
    """Q2 hexahedra: the affine-only validation refuses them (straight or
    not); the general build takes straight and curved cells, refuses a cell
    whose det J turns negative at a Gauss point; the exact reference tensor
    equals the 3 x 3 x 3 Gauss rule's (exact for these integrands) to rounding."""
    m = I.hex27_grid(2, 1, 1)
    assert api.validate_mesh(m.elem, m.coords, m.cells) == -2
    hp = api.host_plan(m.elem, m.coords, m.cells, general=True)
    rp, ci = O.pattern(m.elem, m.n_nodes, m.cells)
    np.testing.assert_array_equal(hp["row_ptr"], rp)
    np.testing.assert_array_equal(hp["col_idx"], ci)
    assert len(ci) == 9 * 17 * 9 * 9
    # the centre node of element 0 pushed through a face: inverted near that face
    c = m.coords.copy()
    centre = m.cells[0, I._HEX27_LATTICE.index((1, 1, 1))]
    assert np.allclose(c[centre], [0.5, 0.5, 0.5])
    c[centre] = [0.5, 0.5, 1.4]
    with pytest.raises(_lib.SoptxError) as e:
        api.host_plan(m.elem, c, m.cells, general=True)
    assert e.value.code == -4
    Ms = api.reference_tensor(I.HEX27, api.REF_SYMBOLIC)
    Mq = api.reference_tensor(I.HEX27, api.REF_QUADRATURE)
    assert Ms.shape == (27, 27, 3, 3)
    assert np.abs(Ms - Mq).max() <= 1e-14 * np.abs(Ms).max()
    assert np.abs(Ms - np.transpose(Ms, (1, 0, 3, 2))).max() == 0.0
    # the library's basis and rule against the oracle's (same node order)
    pts, wts = O.quadrature(I.HEX27)
    Mo = np.zeros((27, 27, 3, 3))
    for xq, wq in zip(pts, wts):
        _, g = O.ref_basis(I.HEX27, xq)
        Mo += wq * np.einsum("im,jn->ijmn", g, g)
    assert np.abs(Ms - Mo).max() <= 1e-14 * np.abs(Mo).max()


def _point_gradient_ke(dim, G):
    """Element matrix (E = 1, nu = 0.3) from the per-point geometry of one
    plan column, G[q] = sqrt(w_q |det J_q|) J_q^-1, with the Gauss points and
    reference gradients the in-LDS assembly uses: the 2-point rule on
    [0, 1]^dim, point q at (1 +- 1/sqrt(3)) / 2 by the bits of q, node k at
    corner k ^ ((k >> 1) & 1); block (i, j) = L(sum_q g_i g_j^T),
    g_k = G^T grad phi_k, L(A) = lam A + mu A^T + mu tr(A) I."""
    nu = 0.3
    lam = nu / ((1 + nu) * (1 - 2 * nu)) if dim == 3 else nu / (1 - nu * nu)
    mu = 1 / (2 * (1 + nu))
    gp, gm = (1 + 1 / np.sqrt(3)) / 2, (1 - 1 / np.sqrt(3)) / 2
    nen = 1 << dim
    ke = np.zeros((dim * nen, dim * nen))
    for q in range(nen):
        g = np.zeros((nen, dim))
        for k in range(nen):
            cb = k ^ ((k >> 1) & 1)
            r = np.ones(dim)
            for m in range(dim):
                for n in range(dim):
                    if n != m:
                        r[m] *= gp if ((cb >> n) & 1) == ((q >> n) & 1) else gm
                if not (cb >> m) & 1:
                    r[m] = -r[m]
            g[k] = G[q].T @ r
        for i in range(nen):
            for j in range(nen):
                P = np.outer(g[i], g[j])
                ke[dim * i:dim * i + dim, dim * j:dim * j + dim] += lam * P + mu * P.T + mu * np.trace(P) * np.eye(dim)
    return ke


@pytest.mark.parametrize("elem,dims,jit,renum,canonical", [
    (I.QUAD4, (7, 5), 0.3, False, False), (I.QUAD4, (40, 13), 0.3, True, True), (I.QUAD4, (7, 5), 0.2, True, False),
    (I.HEX8, (4, 3, 3), 0.3, False, False), (I.HEX8, (4, 3, 3), 0.2, True, True), (I.HEX8, (4, 3, 3), 0.3, True, False)])
def test_point_geometry_gives_element_matrices(elem, dims, jit, renum, canonical):
    """The per-point geometry that the in-LDS general assembly reads (qgeo,
    one column per element, or per element rank in a canonical-order plan),
    with that assembly's point and gradient convention, gives every
    element's matrix as the oracle computes it (a different rule
    parametrisation and code).  Renumbered meshes whose jittered lattice is
    recognised take a canonical-order plan."""
    rng = np.random.default_rng(4)
    m0 = I.quad_grid(*dims) if elem == I.QUAD4 else I.hex_grid(*dims)
    m = I.jitter_interior(m0, jit, rng)
    if renum:
        pn, pe = rng.permutation(m.n_nodes), rng.permutation(m.n_cells)
        coords = np.empty_like(m.coords)
        coords[pn] = m.coords
        m = I.Mesh(m.elem, coords, pn[m.cells[pe]].astype(np.int32))
    hp = api.host_plan(m.elem, m.coords, m.cells, general=True)
    d, nc = m.dim, m.n_cells
    q = hp["qgeo"].reshape(1 << d, d, d, nc)
    cols = hp["elem_by_rank"] if len(hp["elem_by_rank"]) else np.arange(nc)
    assert (len(hp["elem_by_rank"]) > 0) == canonical
    for col in range(nc):
        e = int(cols[col])
        ke = _point_gradient_ke(d, q[:, :, :, col])
        kr = O.element_ke0(elem, m.coords[m.cells[e]])
        assert np.max(np.abs(ke - kr)) <= 1e-13 * np.max(np.abs(kr)), (col, e)
