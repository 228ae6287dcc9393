"""The oracle's multi-threaded variants (the CPU baseline's second row) give
bitwise the serial oracle's results: each stored K value, each s_e and dc_e
and the compliance sum keep their summation order, only the work is split
over threads (row blocks for the assembly, elements for the energies)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2505_02438_amd import inputs as I


def _shuffled(pr, seed):
    m0 = pr.mesh
    rng = np.random.default_rng(seed)
    pn = rng.permutation(m0.n_nodes)
    pe = rng.permutation(m0.n_cells)
    coords = np.empty_like(m0.coords)
    coords[pn] = m0.coords
    cells = pn[m0.cells[pe]].astype(np.int32)
    u = np.empty_like(pr.u)
    u.reshape(-1, m0.dim)[pn] = pr.u.reshape(-1, m0.dim)
    mask = np.empty_like(pr.mask)
    mask.reshape(-1, m0.dim)[pn] = pr.mask.reshape(-1, m0.dim)
    return I.Mesh(m0.elem, coords, cells), pr.rho[pe], u, mask


CASES = [(I.QUAD4, None), (I.TRI3, None), (I.HEX8, None), (I.TET10, None), (I.HEX8, "shuffled"),
         (I.TET10, "shuffled"), (I.HEX8, (9, 7, 6))]


@pytest.mark.parametrize("elem,variant", CASES)
def test_mt_variants_bitwise_equal_serial(elem, variant):
    assert O.threads() >= 1
    if variant == "shuffled":
        pr = I.small_problem(elem, seed=71)
        m, rho, u, mask = _shuffled(pr, 72)
    else:
        pr = I.small_problem(elem, seed=71, dims=variant if isinstance(variant, tuple) else None)
        m, rho, u, mask = pr.mesh, pr.rho, pr.u, pr.mask
    rp, ci = O.pattern(elem, m.n_nodes, m.cells)
    for msk in (None, mask):
        K1 = O.assemble(elem, m.coords, m.cells, rho, rp, ci, mask=msk)
        K2 = O.assemble(elem, m.coords, m.cells, rho, rp, ci, mask=msk, mt=True)
        assert np.array_equal(K1, K2)
    assert np.array_equal(O.element_energy(elem, m.coords, m.cells, u),
                          O.element_energy(elem, m.coords, m.cells, u, mt=True))
    assert np.array_equal(O.sensitivity(elem, m.coords, m.cells, rho, u),
                          O.sensitivity(elem, m.coords, m.cells, rho, u, mt=True))
    f = np.linspace(-1.0, 1.0, m.ndof)
    assert np.array_equal(O.compliance(elem, m.coords, m.cells, rho, u, f),
                          O.compliance(elem, m.coords, m.cells, rho, u, f, mt=True))


def test_mt_assembly_more_threads_than_rows():
    """A mesh of one element: most threads own no row (empty blocks)."""
    pr = I.small_problem(I.QUAD4, seed=73, dims=(1, 1))
    m = pr.mesh
    rp, ci = O.pattern(m.elem, m.n_nodes, m.cells)
    K1 = O.assemble(m.elem, m.coords, m.cells, pr.rho, rp, ci, mask=pr.mask)
    K2 = O.assemble(m.elem, m.coords, m.cells, pr.rho, rp, ci, mask=pr.mask, mt=True)
    assert np.array_equal(K1, K2)
