"""The filter step (Sec. 2.4) on the GPU, through the C ABI, against the
filter oracle: the sensitivity filter, the density filter with the Heaviside
projection, and the density filter's chain rule.

Tolerances: each output is compared with the oracle relative to the sum of
the magnitudes of its terms (sum_j H_ij |x_j| ... over the row), <= 1e-13;
the row sums use another order on the GPU (lanes and an xor tree), so a few
units in the last place per term are expected.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import filters as OF
from paper_2505_02438_amd import api
from paper_2505_02438_amd import inputs as I

from gpu_util import dev, host

pytestmark = pytest.mark.gpu
TOL = 1e-13


def _case(elem, rmin, seed, mesh=None):
    m = mesh if mesh is not None else I.small_problem(elem, seed=seed).mesh
    flt = api.Filter(m.elem, m.coords, m.cells, rmin)
    c = OF.centroids(m.elem, m.coords, m.cells)
    v = OF.volumes(m.elem, m.coords, m.cells)
    H = OF.filter_matrix(c, rmin)
    rng = np.random.default_rng(seed)
    return m, flt, H, v, rng


def _scaled(got, ref, scale):
    scale = np.where(scale > 0, scale, 1.0)
    return float(np.max(np.abs(got - ref) / scale)) if len(ref) else 0.0


CASES = [(I.QUAD4, 1.5), (I.QUAD4, 6.0), (I.TRI3, 2.0), (I.HEX8, 1.5), (I.HEX8, 2.6), (I.TET10, 1.2)]


@pytest.mark.parametrize("elem,rmin", CASES)
def test_filter_upload_and_products(elem, rmin):
    m, flt, H, v, rng = _case(elem, rmin, 31)
    rp, col, w, vol = flt.matrix()
    hh = api.filter_matrix_host(elem, m.coords, m.cells, rmin)
    assert np.array_equal(rp, hh["row_ptr"]) and np.array_equal(col, hh["col"])
    assert np.array_equal(w, hh["w"]) and np.array_equal(vol, hh["vol"])
    n = flt.n
    rho = rng.uniform(1e-4, 1.0, n)
    rho[:: 7] = 1e-4                                  # below gamma: max(gamma, rho) = gamma
    dc = -rng.exponential(1.0, n)
    # sensitivity filter
    got = host(flt.sensitivity(dev(rho), dev(dc)))
    ref = OF.sensitivity_filter(H, rho, dc)
    scale = OF.h_product(H, np.abs(rho * dc)) / (np.maximum(OF.GAMMA, rho) * OF.h_product(H, np.ones(n)))
    e_s = _scaled(got, ref, scale)
    # density filter and projection
    for beta in (None, 0.0, 1.0, 8.0, 64.0):
        out = flt.density(dev(rho), beta=beta)
        rt = host(out if beta is None else out[0])
        ref_t = OF.density_filter(H, v, rho)
        e_d = _scaled(rt, ref_t, ref_t)
        assert e_d <= TOL, (beta, e_d)
        if beta is not None:
            rb = host(out[1])
            ref_b = OF.heaviside(rt, beta)                 # same rho~: the projection alone
            assert float(np.max(np.abs(rb - ref_b))) <= 1e-15 * max(1.0, beta), beta
            assert float(np.max(np.abs(rb - OF.heaviside(ref_t, beta)))) <= 1e-13 * max(1.0, beta)
    # chain rule, without and with the projection
    g = rng.standard_normal(n)
    gb = host(flt.density_backward(dev(g)))
    ref_g = OF.density_filter_backward(H, v, g)
    sc_g = OF.density_filter_backward(H, v, np.abs(g))
    e_b = _scaled(gb, ref_g, sc_g)
    rt = OF.density_filter(H, v, rho)
    beta = 4.0
    gh = host(flt.density_backward(dev(g), rho_tilde=dev(rt), beta=beta))
    gt = g * OF.heaviside_grad(rt, beta)
    ref_h = OF.density_filter_backward(H, v, gt)
    e_h = _scaled(gh, ref_h, OF.density_filter_backward(H, v, np.abs(gt)))
    print(f"elem={elem} rmin={rmin} n={n} nnz={flt.nnz} lanes={flt.lanes}: sens {e_s:.1e} bwd {e_b:.1e} "
          f"bwd+heaviside {e_h:.1e}")
    assert e_s <= TOL and e_b <= TOL and e_h <= TOL


@pytest.mark.parametrize("rmin", [1.2, 2.5, 4.0, 6.0, 10.0])
def test_every_lane_width(rmin):
    """Radii whose mean row lengths select 4, 8, 16, 32 and 64 lanes per row, on
    a grid whose element count is not a multiple of the rows per block."""
    m = I.quad_grid(37, 23)
    _, flt, H, v, rng = _case(I.QUAD4, rmin, 32, mesh=m)
    rho = rng.uniform(0.0, 1.0, flt.n)
    dc = -rng.exponential(1.0, flt.n)
    ref = OF.sensitivity_filter(H, rho, dc)
    scale = OF.h_product(H, np.abs(rho * dc)) / (np.maximum(OF.GAMMA, rho) * OF.h_product(H, np.ones(flt.n)))
    e_s = _scaled(host(flt.sensitivity(dev(rho), dev(dc))), ref, scale)
    ref_t = OF.density_filter(H, v, rho)
    e_d = _scaled(host(flt.density(dev(rho))), ref_t, OF.density_filter(H, v, np.abs(rho)))
    g = rng.standard_normal(flt.n)
    e_b = _scaled(host(flt.density_backward(dev(g))), OF.density_filter_backward(H, v, g),
                  OF.density_filter_backward(H, v, np.abs(g)))
    print(f"rmin={rmin} lanes={flt.lanes} mean row {flt.nnz / flt.n:.1f}: {e_s:.1e} {e_d:.1e} {e_b:.1e}")
    assert max(e_s, e_d, e_b) <= TOL


def test_lane_widths_cover_all_variants():
    m = I.quad_grid(37, 23)
    lanes = {api.Filter(m.elem, m.coords, m.cells, r).lanes for r in (1.2, 2.5, 4.0, 6.0, 10.0)}
    assert lanes == {4, 8, 16, 32, 64}


def test_filter_deterministic_and_degenerate():
    m, flt, H, v, rng = _case(I.HEX8, 1.5, 33)
    rho = dev(rng.uniform(0, 1, flt.n))
    a, b = flt.density(rho, beta=2.0), flt.density(rho, beta=2.0)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    g = dev(rng.standard_normal(flt.n))
    assert torch.equal(flt.density_backward(g), flt.density_backward(g))
    # constant design: the density filter returns it exactly up to rounding
    c = flt.density(torch.full_like(rho, 0.3))
    assert float(torch.max(torch.abs(c - 0.3))) <= 1e-15
    # aliasing an output onto an input is refused
    with pytest.raises(api._lib.SoptxError):
        flt.density(rho, rho_tilde=rho)
    # a mesh with no elements: a valid empty filter, calls are no-ops
    e = I.quad_grid(2, 2)
    f0 = api.Filter(e.elem, e.coords, e.cells[:0], 1.5)
    assert f0.n == 0 and f0.nnz == 0
    z = torch.empty(0, dtype=torch.float64, device="cuda")
    f0.density(z, beta=1.0)
    f0.sensitivity(z, z)
    f0.density_backward(z)


def test_filter_full_cantilever_sampled_rows():
    """The 120 x 40 x 40 hexahedra at the 3D cantilever's radius 1.5: sampled
    rows against the oracle's rows computed one by one, and properties that
    hold on every row."""
    pr = I.cantilever_hex()
    m = pr.mesh
    flt = api.Filter.from_mesh(m, 1.5)
    n = flt.n
    assert n == 192000
    c = OF.centroids(m.elem, m.coords, m.cells)
    v = OF.volumes(m.elem, m.coords, m.cells)
    rng = np.random.default_rng(34)
    rho = rng.uniform(1e-3, 1.0, n)
    dc = -rng.exponential(1.0, n)
    g = rng.standard_normal(n)
    d_rho = dev(rho)
    rt, rb = flt.density(d_rho, beta=8.0)
    rt, rb = host(rt), host(rb)
    dcf = host(flt.sensitivity(d_rho, dev(dc)))
    gb = host(flt.density_backward(dev(g), rho_tilde=dev(rt), beta=8.0))
    rows = np.unique(np.concatenate([rng.integers(0, n, 24), [0, n - 1, 40 * 40 * 60 + 20 * 40 + 20]]))
    for i, (cj, wj) in zip(rows, OF.filter_rows(c, 1.5, rows)):
        hsv = float(wj @ v[cj])
        ref_t = float(wj @ (v[cj] * rho[cj])) / hsv
        assert abs(rt[i] - ref_t) <= TOL * ref_t
        assert abs(rb[i] - OF.heaviside(np.array([ref_t]), 8.0)[0]) <= 1e-12
        num = float(wj @ (rho[cj] * dc[cj]))
        ref_s = num / (max(OF.GAMMA, rho[i]) * float(wj.sum()))
        assert abs(dcf[i] - ref_s) <= TOL * abs(float(wj @ np.abs(rho[cj] * dc[cj])) / (max(OF.GAMMA, rho[i]) * wj.sum()))
        # chain rule at row i needs t_k = g_k h'(rho~_k) / hsv_k of its neighbours k
        nbr = OF.filter_rows(c, 1.5, cj)
        t = np.array([g[k] * OF.heaviside_grad(np.array([rt[k]]), 8.0)[0] / float(wk @ v[ck])
                      for k, (ck, wk) in zip(cj, nbr)])
        ref_b = v[i] * float(wj @ t)
        assert abs(gb[i] - ref_b) <= TOL * v[i] * float(wj @ np.abs(t))
    # every row: 19 neighbours inside, fewer on faces, edges and corners
    rp, _, _, _ = flt.matrix()
    cnt = np.diff(rp)
    assert cnt.max() == 19 and cnt.min() == 1 + 3 + 3 and flt.nnz == int(cnt.sum())
    # a constant design is reproduced on every row
    k = host(flt.density(torch.full_like(d_rho, 0.3)))
    assert float(np.max(np.abs(k - 0.3))) <= 1e-15
