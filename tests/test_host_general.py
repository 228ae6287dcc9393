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
