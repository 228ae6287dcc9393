"""Host side of the filter step (Sec. 2.4): the filter matrix H, the element
measures and the row sums that soptx_build_filter uploads, built on the host
by the library's uniform-cell search, against the oracle's brute-force
construction; the argument checks of the filter entry points.  No GPU."""
import ctypes

import numpy as np
import pytest

from oracle import filters as OF
from paper_2505_02438_amd import _lib, api
from paper_2505_02438_amd import inputs as I

CASES = [(I.QUAD4, 1.5), (I.QUAD4, 6.0), (I.TRI3, 2.0), (I.HEX8, 1.5), (I.HEX8, 2.6), (I.TET10, 1.2)]


def _oracle(elem, m, rmin):
    c = OF.centroids(elem, m.coords, m.cells)
    v = OF.volumes(elem, m.coords, m.cells)
    H = OF.filter_matrix(c, rmin)
    return H, v


@pytest.mark.parametrize("elem,rmin", CASES)
def test_filter_matrix_matches_oracle(elem, rmin):
    m = I.small_problem(elem, seed=21).mesh
    got = api.filter_matrix_host(elem, m.coords, m.cells, rmin)
    (rp, col, w), v = _oracle(elem, m, rmin)
    # the neighbour sets and their order: exact
    np.testing.assert_array_equal(got["row_ptr"], rp)
    np.testing.assert_array_equal(got["col"], col)
    # weights: the same operations on the same centroids
    np.testing.assert_allclose(got["w"], w, rtol=1e-15, atol=0)
    np.testing.assert_allclose(got["vol"], v, rtol=1e-13, atol=0)
    np.testing.assert_allclose(got["hsv"], OF.h_product((rp, col, w), v), rtol=1e-14)
    np.testing.assert_allclose(got["hs"], OF.h_product((rp, col, w), np.ones(len(v))), rtol=1e-14)


def test_filter_matrix_larger_grid_and_radius_edge():
    """A radius equal to a neighbour distance keeps that neighbour out (H = 0),
    and a radius far above the domain's size puts every element in every row."""
    m = I.quad_grid(20, 10)
    got = api.filter_matrix_host(I.QUAD4, m.coords, m.cells, 1.0)
    assert np.all(np.diff(got["row_ptr"]) == 1)          # distance 1 exactly: only the element itself
    got = api.filter_matrix_host(I.QUAD4, m.coords, m.cells, 100.0)
    assert np.all(np.diff(got["row_ptr"]) == 200)
    mh = I.hex_grid(12, 7, 5)
    got = api.filter_matrix_host(I.HEX8, mh.coords, mh.cells, 1.5)
    (rp, col, w), _ = _oracle(I.HEX8, mh, 1.5)
    np.testing.assert_array_equal(got["row_ptr"], rp)
    np.testing.assert_array_equal(got["col"], col)


def test_filter_matrix_tiny_radius_many_cells():
    """A radius tiny against the domain: the cell grid is coarsened (bounded
    memory) and each row holds only its element."""
    m = I.quad_grid(30, 30, h=1000.0)
    got = api.filter_matrix_host(I.QUAD4, m.coords, m.cells, 1e-3)
    assert np.all(np.diff(got["row_ptr"]) == 1) and np.all(got["w"] == 1e-3)


def _renumber(m, order):
    """The same mesh with its elements listed in another order."""
    return I.Mesh(m.elem, m.coords, np.ascontiguousarray(m.cells[order]))


def test_stencil_form_detection():
    """The stencil form is found on structured grids in any lexicographic
    numbering, with the grid sizes in numbering order, and refused where rows
    differ (sheared or shuffled meshes, weights differing in the last bit,
    more than 512 offsets)."""
    m = I.quad_grid(37, 23)
    assert api.filter_stencil_host(m.elem, m.coords, m.cells, 1.5) == (9, (1, 37, 23))
    assert api.filter_stencil_host(m.elem, m.coords, m.cells, 6.0)[0] == 109
    h = I.hex_grid(9, 7, 5)
    assert api.filter_stencil_host(h.elem, h.coords, h.cells, 1.5) == (19, (9, 7, 5))
    # x fastest instead of slowest: found with the axes swapped
    ei, ej = np.meshgrid(np.arange(37), np.arange(23), indexing="ij")
    order = np.lexsort((ei.ravel(), ej.ravel()))          # sort by j, then i
    mt = _renumber(m, order)
    assert api.filter_stencil_host(mt.elem, mt.coords, mt.cells, 1.5) == (9, (1, 23, 37))
    # a shuffled numbering, triangles, a sheared grid: no stencil
    rng = np.random.default_rng(1)
    ms = _renumber(m, rng.permutation(m.n_cells))
    assert api.filter_stencil_host(ms.elem, ms.coords, ms.cells, 1.5)[0] == 0
    t = I.small_problem(I.TRI3, seed=3).mesh
    assert api.filter_stencil_host(t.elem, t.coords, t.cells, 2.0)[0] == 0
    sk = I.skew_mesh(I.quad_grid(9, 6), "global")
    assert api.filter_stencil_host(sk.elem, sk.coords, sk.cells, 1.5)[0] == 0
    # spacing 0.1: centroid differences, hence weights, vary in the last bit
    m1 = I.quad_grid(30, 20, h=0.1)
    assert api.filter_stencil_host(m1.elem, m1.coords, m1.cells, 0.15)[0] == 0
    # rows of up to 2,809 offsets: over the cap
    big = I.quad_grid(60, 60)
    assert api.filter_stencil_host(big.elem, big.coords, big.cells, 30.0)[0] == 0
    # the stencil is the matrix: every row's entries are its in-grid offsets
    hh = api.filter_matrix_host(h.elem, h.coords, h.cells, 1.5)
    assert hh["row_ptr"][-1] == 19 * 9 * 7 * 5 - 2 * (7 * 5 * (1 + 4) + 9 * 5 * (1 + 4) + 9 * 7 * (1 + 4)) + \
        4 * (9 + 7 + 5)


def test_filter_argument_errors():
    m = I.quad_grid(3, 2)
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(_lib.SoptxError) as e:
            api.filter_matrix_host(I.QUAD4, m.coords, m.cells, bad)
        assert e.value.code == -1
    cells = m.cells.copy()
    cells[0, 1] = 999
    with pytest.raises(_lib.SoptxError) as e:
        api.filter_matrix_host(I.QUAD4, m.coords, cells, 1.5)
    assert e.value.code == -3
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.soptx_build_filter(None, 1.5, ctypes.byref(h), None) == -1
    assert L.soptx_filter_sensitivity(None, None, None, None, None) == -1
    assert L.soptx_filter_density(None, None, 1.0, None, None, None) == -1
    assert L.soptx_filter_density_backward(None, None, 1.0, None, None, None) == -1
    n, nnz = ctypes.c_int64(), ctypes.c_int64()
    assert L.soptx_filter_info(None, ctypes.byref(n), ctypes.byref(nnz), None) == -1
    L.soptx_destroy_filter(None)


def test_oc_argument_errors():
    """soptx_oc_update rejects bad parameters before touching the device."""
    L = _lib.lib()
    res = _lib.OcResult()
    good = dict(move=0.2, eta=0.5, lmax=1e9, tol=1e-3, max_steps=200)
    bad = [dict(move=0.0), dict(move=1.5), dict(eta=0.0), dict(eta=1.2), dict(lmax=0.0), dict(lmax=float("inf")),
           dict(tol=0.0), dict(tol=1.0), dict(max_steps=0), dict(max_steps=1001)]
    for b in bad:
        p = _lib.OcParams(**{**good, **b})
        assert L.soptx_oc_update(10, 8, 8, 8, 1.0, ctypes.byref(p), 16, ctypes.byref(res), None) == -1, b
    p = _lib.OcParams(**good)
    assert L.soptx_oc_update(-1, None, None, None, 1.0, ctypes.byref(p), None, ctypes.byref(res), None) == -1
    assert L.soptx_oc_update(10, None, None, None, 1.0, ctypes.byref(p), None, ctypes.byref(res), None) == -1
    assert L.soptx_oc_update(10, 8, 8, 8, float("nan"), ctypes.byref(p), 16, ctypes.byref(res), None) == -1
    assert L.soptx_oc_update(10, 8, 8, 8, 1.0, None, 16, ctypes.byref(res), None) == -1
    assert L.soptx_oc_update(10, 8, 8, 8, 1.0, ctypes.byref(p), 8, ctypes.byref(res), None) == -1   # aliasing
    # n = 0: nothing runs, a zero result
    assert L.soptx_oc_update(0, None, None, None, 1.0, ctypes.byref(p), None, ctypes.byref(res), None) == 0
    assert res.steps == 0 and res.lambda_ == 0.0


def test_heaviside_beta_continuation():
    assert api.heaviside_beta(0) == 1.0 and api.heaviside_beta(49) == 1.0 and api.heaviside_beta(50) == 2.0
    assert api.heaviside_beta(50 * 9) == 512.0 and api.heaviside_beta(10 ** 6) == 512.0
    with pytest.raises(ValueError):
        api.heaviside_beta(-1)


@pytest.mark.parametrize("elem", [I.QUAD4, I.HEX8, I.HEX27])
def test_filter_on_general_q1(elem):
    """Non-affine Q1 cells and curved Q2 hexahedra are accepted; their
    measures are the Gauss-rule integral of |det J| (the oracle's definition)
    and tile the box; centroids are the means of the corner nodes."""
    m0 = {I.QUAD4: lambda: I.quad_grid(9, 7), I.HEX8: lambda: I.hex_grid(4, 3, 3),
          I.HEX27: lambda: I.hex27_grid(4, 3, 3)}[elem]()
    m = I.jitter_interior(m0, 0.12 if elem == I.HEX27 else 0.3, np.random.default_rng(2))
    hh = api.filter_matrix_host(m.elem, m.coords, m.cells, 1.6)
    v = OF.volumes(elem, m.coords, m.cells)
    np.testing.assert_allclose(hh["vol"], v, rtol=1e-14)
    assert abs(hh["vol"].sum() - (63.0 if elem == I.QUAD4 else 36.0)) <= 1e-12
    (rp, col, w), _ = _oracle(elem, m, 1.6)
    np.testing.assert_array_equal(hh["row_ptr"], rp)
    np.testing.assert_array_equal(hh["col"], col)
