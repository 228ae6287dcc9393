"""Assembly with per-quadrature-point geometry (soptx_assemble_general) on
the GPU, through the C ABI: general (non-affine) Q1 quadrilaterals and
hexahedra against the oracle's assembly (row-scaled error, the C12 metric,
<= 1e-12), with and without Dirichlet rows; on affine meshes against the
separated-form kernel (two different formulas, same matrix); determinism;
the affine-only calls refuse a non-affine handle; the full 120x40x40
hexahedral cantilever with jittered interior nodes against the oracle."""
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
    mat = api.Material(E0=pr.E0, Emin=pr.Emin, nu=pr.nu, p=pr.p)
    K = host(pat.assemble_general(mat, dev(pr.rho), dev(pr.mask)))
    rp, ci = O.pattern(m.elem, m.n_nodes, m.cells)
    Kr = O.assemble(m.elem, m.coords, m.cells, pr.rho, rp, ci, mask=pr.mask)
    err = _row_scaled(rp, K, Kr)
    print(f"full 120x40x40 jittered hex: row-scaled {err:.1e}")
    assert err <= 1e-12
