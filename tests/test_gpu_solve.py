"""The equilibrium solve K u = f (Sec. 2.2) on the assembled CSR values:
soptx_spmv and the preconditioned CG soptx_pcg (the solver module's
iterative solver, Sec. 3.2), through the C ABI.

* SpMV against the oracle's CSR product, row by row (scaled by sum |K| |x|);
* CG against the oracle's banded Cholesky solve on small meshes of every
  element type and on the 60 x 20 MBB beam: the true residual
  ||f - K u|| / ||f|| (oracle product) and the solution;
* bitwise reproducible, a zero right-hand side needs no iteration;
* the full 3D cantilever (120 x 40 x 40 Q1 hex) solved to a small true
  residual, where f^T u = u^T K u (Eq. cmpd) then holds.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2505_02438_amd import api
from paper_2505_02438_amd import inputs as I

from gpu_util import dev, host

pytestmark = pytest.mark.gpu
ELEMS = [I.QUAD4, I.TRI3, I.HEX8, I.TET10]


def _system(pr):
    m = pr.mesh
    pat = api.Pattern.from_mesh(m)
    mat = api.Material(E0=pr.E0, Emin=pr.Emin, nu=pr.nu, p=pr.p)
    K = pat.assemble(mat, dev(pr.rho), dev(pr.mask))
    rp, ci = O.pattern(m.elem, m.n_nodes, m.cells)
    return pat, mat, K, rp, ci


@pytest.mark.parametrize("elem", ELEMS)
def test_spmv_matches_oracle(elem):
    pr = I.small_problem(elem, seed=71)
    pat, _, K, rp, ci = _system(pr)
    x = np.random.default_rng(72).standard_normal(pr.mesh.ndof)
    y = host(pat.spmv(K, dev(x)))
    Kh = host(K)
    ref = O.spmv(rp, ci, Kh, x)
    scale = O.spmv(rp, ci, np.abs(Kh), np.abs(x))
    err = float(np.max(np.abs(y - ref) / scale))
    print(f"elem={elem} spmv scaled err {err:.2e}")
    assert err <= 1e-14


def _check_solve(pr, rtol, tol_res, tol_u, manufactured=False):
    pat, _, K, rp, ci = _system(pr)
    Kh = host(K)
    # manufactured: f = K u_true for the seeded u (zero on the fixed dofs, so
    # f is too); otherwise the problem's own load
    f = O.spmv(rp, ci, Kh, pr.u) if manufactured else pr.f
    assert np.any(f != 0) and np.all(f[pr.mask != 0] == 0)
    u, iters, rel = pat.pcg(K, dev(f), rtol=rtol, max_iter=20000)
    uh = host(u)
    res = np.linalg.norm(f - O.spmv(rp, ci, Kh, uh)) / np.linalg.norm(f)
    uref = O.solve(rp, ci, Kh, f)
    uerr = np.linalg.norm(uh - uref) / np.linalg.norm(uref)
    print(f"{pr.name}: {iters} iterations, recurrence {rel:.1e}, true residual {res:.1e}, |u - u_direct| {uerr:.1e}")
    assert rel <= rtol and res <= tol_res and uerr <= tol_u
    return pat, K, f, uh


@pytest.mark.parametrize("elem", ELEMS)
def test_pcg_matches_direct_solve(elem):
    pr = I.small_problem(elem, seed=73)
    _, _, _, uh = _check_solve(pr, 1e-12, 1e-10, 1e-6, manufactured=True)
    assert np.linalg.norm(uh - pr.u) <= 1e-6 * np.linalg.norm(pr.u)


def test_pcg_mbb_beam_against_direct_solve():
    _check_solve(I.mbb_q1(), 1e-12, 1e-10, 1e-6)


def test_pcg_deterministic_and_zero_rhs():
    pr = I.small_problem(I.HEX8, seed=74)
    pat, _, K, rp, ci = _system(pr)
    f = dev(pr.f)
    u1, it1, r1 = pat.pcg(K, f, rtol=1e-10)
    u2, it2, r2 = pat.pcg(K, f, rtol=1e-10)
    assert it1 == it2 and r1 == r2 and torch.equal(u1, u2)
    z, it0, r0 = pat.pcg(K, torch.zeros_like(f))
    assert it0 == 0 and r0 == 0.0 and not torch.any(z)
    # the initial guess is used: with f = K u_true from the same product, a
    # start at u_true has a zero residual, so no iteration and u is untouched
    ut = dev(pr.u)
    fm = pat.spmv(K, ut)
    u3, it3, r3 = pat.pcg(K, fm, u=ut.clone(), rtol=1e-10)
    assert it3 == 0 and r3 == 0.0 and torch.equal(u3, ut)


def test_pcg_full_cantilever_hex():
    pr = I.cantilever_hex()
    pat, mat, K, _, _ = _system(pr)
    f = dev(pr.f)
    u, iters, rel = pat.pcg(K, f, rtol=1e-9, max_iter=20000)
    r = f - pat.spmv(K, u)
    res = float(torch.linalg.norm(r) / torch.linalg.norm(f))
    _, c = pat.evaluate(mat, dev(pr.rho), u, f=f)
    c = host(c)
    print(f"3D cantilever: {iters} iterations, recurrence {rel:.1e}, true residual {res:.1e}, "
          f"u^T K u {c[0]:.10g}, f^T u {c[1]:.10g}")
    assert rel <= 1e-9 and res <= 1e-8
    assert abs(c[0] - c[1]) <= 1e-7 * abs(c[1])
