"""Pins of the filter oracle (Sec. 2.4) against facts other than itself:
an independent neighbourhood search (scipy's KD-tree, the structure the
paper names for building H), hand-computed rows on a uniform grid, closed
forms for element measures, invariants of the filters (constants and, on
interior rows, linear fields are reproduced), the adjoint identity of the
density filter's chain rule, finite differences of the Heaviside chain, and
the limits of the projection.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import filters as F
from paper_2505_02438_amd import inputs as I


def _dense(H, n):
    row_ptr, col, w = H
    A = np.zeros((n, n))
    for i in range(n):
        for k in range(row_ptr[i], row_ptr[i + 1]):
            A[i, col[k]] = w[k]
    return A


@pytest.mark.parametrize("elem,rmin", [(I.QUAD4, 1.5), (I.QUAD4, 3.2), (I.TRI3, 2.0), (I.HEX8, 1.5),
                                       (I.TET10, 1.1)])
def test_filter_matrix_matches_kdtree(elem, rmin):
    m = I.small_problem(elem, seed=5).mesh
    c = F.centroids(elem, m.coords, m.cells)
    H = F.filter_matrix(c, rmin, block=97)          # a block size that leaves a ragged tail
    n = c.shape[0]
    tree = cKDTree(c)
    D = tree.sparse_distance_matrix(tree, rmin, output_type="coo_matrix").tocsr()
    D.sort_indices()
    ref = np.zeros((n, n))
    r, cc = D.nonzero()
    ref[r, cc] = rmin - np.asarray(D[r, cc]).ravel()
    ref[np.arange(n), np.arange(n)] = rmin          # the zero self-distance is not stored by scipy
    ref[ref < 0] = 0.0
    A = _dense(H, n)
    assert np.array_equal(A > 0, ref > 0)
    np.testing.assert_allclose(A, ref, rtol=0, atol=1e-13)
    # symmetric, ascending columns, positive weights, the diagonal is rmin
    assert np.array_equal(A, A.T)
    row_ptr, col, w = H
    for i in range(n):
        seg = col[row_ptr[i]:row_ptr[i + 1]]
        assert np.all(np.diff(seg) > 0) and i in seg
    assert np.all(w > 0)
    assert np.all(np.diag(A) == rmin)


def test_filter_rows_match_whole_matrix():
    m = I.small_problem(I.TRI3, seed=8).mesh
    c = F.centroids(I.TRI3, m.coords, m.cells)
    row_ptr, col, w = F.filter_matrix(c, 2.2)
    rows = [0, 5, len(c) - 1]
    for i, (cj, wj) in zip(rows, F.filter_rows(c, 2.2, rows)):
        np.testing.assert_array_equal(cj, col[row_ptr[i]:row_ptr[i + 1]])
        np.testing.assert_array_equal(wj, w[row_ptr[i]:row_ptr[i + 1]])


def test_filter_row_on_uniform_grid_by_hand():
    """Unit squares, r_min = 1.5: an interior row holds the element (1.5), its
    4 edge neighbours (0.5) and 4 diagonal ones (1.5 - sqrt 2); the next ring
    (distance 2) is outside."""
    m = I.quad_grid(7, 6)
    c = F.centroids(I.QUAD4, m.coords, m.cells)
    row_ptr, col, w = F.filter_matrix(c, 1.5)
    i = 3 * 6 + 3                                    # element (3, 3), interior (index ei ny + ej)
    seg = w[row_ptr[i]:row_ptr[i + 1]]
    assert len(seg) == 9
    assert sorted(seg.tolist()) == sorted([1.5] + [0.5] * 4 + [1.5 - np.sqrt(2.0)] * 4)
    i0 = 0                                           # corner: itself, 2 edge, 1 diagonal
    assert row_ptr[i0 + 1] - row_ptr[i0] == 4
    # 3D unit cubes, r = 1.5 (the 3D cantilever's radius): 1 + 6 + 12 = 19 neighbours inside
    mh = I.hex_grid(5, 5, 5)
    ch = F.centroids(I.HEX8, mh.coords, mh.cells)
    rp, _, wh = F.filter_matrix(ch, 1.5)
    k = (2 * 5 + 2) * 5 + 2                          # element (2, 2, 2)
    assert rp[k + 1] - rp[k] == 19
    assert abs(wh[rp[k]:rp[k + 1]].sum() - (1.5 + 6 * 0.5 + 12 * (1.5 - np.sqrt(2.0)))) < 1e-14


def test_centroids_and_volumes_closed_forms():
    m = I.quad_grid(3, 2, h=0.5)
    np.testing.assert_allclose(F.volumes(I.QUAD4, m.coords, m.cells), 0.25, rtol=1e-15)
    np.testing.assert_allclose(F.centroids(I.QUAD4, m.coords, m.cells)[0], [0.25, 0.25], rtol=0, atol=1e-16)
    mh = I.hex_grid(2, 2, 2, h=2.0)
    np.testing.assert_allclose(F.volumes(I.HEX8, mh.coords, mh.cells), 8.0, rtol=1e-15)
    # jittered triangles: the shoelace formula
    mt = I.tri_grid(4, 3, jitter=0.2, rng=np.random.default_rng(3))
    x = mt.coords[mt.cells]
    shoe = 0.5 * np.abs((x[:, 1, 0] - x[:, 0, 0]) * (x[:, 2, 1] - x[:, 0, 1])
                        - (x[:, 2, 0] - x[:, 0, 0]) * (x[:, 1, 1] - x[:, 0, 1]))
    np.testing.assert_allclose(F.volumes(I.TRI3, mt.coords, mt.cells), shoe, rtol=1e-13)
    assert abs(F.volumes(I.TRI3, mt.coords, mt.cells).sum() - 4 * 3) < 1e-12   # they tile the box
    # P2 tets of a jittered box tile it too; the centroid is the vertex mean
    pr = I.small_problem(I.TET10, seed=9)
    v = F.volumes(I.TET10, pr.mesh.coords, pr.mesh.cells)
    x = pr.mesh.coords[pr.mesh.cells[:, :4]]
    vol6 = np.abs(np.einsum("ej,ej->e", x[:, 1] - x[:, 0], np.cross(x[:, 2] - x[:, 0], x[:, 3] - x[:, 0])))
    np.testing.assert_allclose(v, vol6 / 6.0, rtol=1e-12)
    np.testing.assert_allclose(F.centroids(I.TET10, pr.mesh.coords, pr.mesh.cells), x.mean(axis=1),
                               rtol=0, atol=1e-14)


def test_sensitivity_filter_worked_example():
    """Three unit elements in a row, r_min = 1.5: H = [[1.5, .5, 0], [.5, 1.5, .5], [0, .5, 1.5]]."""
    c = np.array([[0.5, 0.5], [1.5, 0.5], [2.5, 0.5]])
    H = F.filter_matrix(c, 1.5)
    np.testing.assert_array_equal(_dense(H, 3), [[1.5, 0.5, 0], [0.5, 1.5, 0.5], [0, 0.5, 1.5]])
    rho = np.array([1.0, 0.5, 1e-4])
    dc = np.array([-2.0, -4.0, -8.0])
    got = F.sensitivity_filter(H, rho, dc)
    exp0 = (1.5 * 1.0 * -2.0 + 0.5 * 0.5 * -4.0) / (1.0 * 2.0)
    exp1 = (0.5 * -2.0 + 1.5 * 0.5 * -4.0 + 0.5 * 1e-4 * -8.0) / (0.5 * 2.5)
    exp2 = (0.5 * 0.5 * -4.0 + 1.5 * 1e-4 * -8.0) / (1e-3 * 2.0)    # gamma = 1e-3 takes over
    np.testing.assert_allclose(got, [exp0, exp1, exp2], rtol=1e-15)
    # rho = 1 and constant dc: unchanged
    np.testing.assert_allclose(F.sensitivity_filter(H, np.ones(3), np.full(3, -3.0)), -3.0, rtol=1e-15)


def test_density_filter_invariants():
    m = I.quad_grid(12, 9)
    c = F.centroids(I.QUAD4, m.coords, m.cells)
    v = F.volumes(I.QUAD4, m.coords, m.cells)
    H = F.filter_matrix(c, 2.5)
    np.testing.assert_allclose(F.density_filter(H, v, np.full(len(v), 0.37)), 0.37, rtol=1e-15)
    # a linear field is reproduced on rows whose disc lies inside the mesh
    lin = 0.1 + 0.03 * c[:, 0] - 0.02 * c[:, 1]
    out = F.density_filter(H, v, lin)
    inner = (c[:, 0] > 2.5) & (c[:, 0] < 12 - 2.5) & (c[:, 1] > 2.5) & (c[:, 1] < 9 - 2.5)
    assert inner.sum() >= 8
    np.testing.assert_allclose(out[inner], lin[inner], rtol=1e-14)
    # a convex combination: bounded by the input's range
    rho = np.random.default_rng(2).uniform(0.1, 0.9, len(v))
    out = F.density_filter(H, v, rho)
    assert out.min() >= rho.min() and out.max() <= rho.max()


@pytest.mark.parametrize("elem", [I.QUAD4, I.TRI3, I.HEX8])
def test_density_filter_backward_is_the_adjoint(elem):
    """<F rho, g> = <rho, F^T g> with F the density filter (a linear map); a
    transposed weight or a misplaced v_j breaks it on non-uniform meshes."""
    m = I.small_problem(elem, seed=11).mesh
    c = F.centroids(elem, m.coords, m.cells)
    v = F.volumes(elem, m.coords, m.cells)
    H = F.filter_matrix(c, 1.7)
    rng = np.random.default_rng(12)
    rho, g = rng.uniform(0, 1, len(v)), rng.standard_normal(len(v))
    lhs = float(F.density_filter(H, v, rho) @ g)
    rhs = float(rho @ F.density_filter_backward(H, v, g))
    assert abs(lhs - rhs) <= 1e-13 * (np.abs(rho) @ np.abs(F.density_filter_backward(H, v, np.abs(g))))
    # and against the dense matrix of the map, column by column
    n = len(v)
    Fm = np.stack([F.density_filter(H, v, e) for e in np.eye(n)], axis=1)
    np.testing.assert_allclose(F.density_filter_backward(H, v, g), Fm.T @ g, rtol=1e-12, atol=1e-15)


def test_heaviside_limits_and_chain_rule():
    rt = np.linspace(0.0, 1.0, 11)
    np.testing.assert_allclose(F.heaviside(rt, 1e-12), rt, atol=1e-11)       # beta -> 0: identity
    for beta in (1.0, 8.0, 512.0):
        hb = F.heaviside(np.array([0.0, 1.0]), beta)
        assert hb[0] == 0.0 and abs(hb[1] - 1.0) <= 1e-15
    assert abs(F.heaviside(np.array([0.5]), 1.0)[0] - (1 - np.exp(-0.5) + 0.5 * np.exp(-1.0))) < 1e-16
    # chain rule through filter and projection, by central differences
    m = I.quad_grid(6, 5)
    c = F.centroids(I.QUAD4, m.coords, m.cells)
    v = F.volumes(I.QUAD4, m.coords, m.cells)
    H = F.filter_matrix(c, 1.8)
    rng = np.random.default_rng(4)
    rho, wgt = rng.uniform(0.2, 0.8, len(v)), rng.standard_normal(len(v))
    beta = 4.0

    def psi(r):
        return float(wgt @ F.heaviside(F.density_filter(H, v, r), beta))

    rt = F.density_filter(H, v, rho)
    grad = F.density_filter_backward(H, v, wgt * F.heaviside_grad(rt, beta))
    h = 1e-6
    for j in (0, 7, 29):
        e = np.zeros(len(v))
        e[j] = h
        fd = (psi(rho + e) - psi(rho - e)) / (2 * h)
        assert abs(fd - grad[j]) <= 1e-7 * max(1.0, abs(grad[j]))
