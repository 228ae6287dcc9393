"""The OC update (Sec. 2.3, Algorithm 1) on the GPU, through the C ABI,
against the OC oracle; and whole optimisation iterations (assembly, CG
solve, sensitivities, filter, OC update, all on the GPU) against the same
iterations run by the oracles.

The device bisection takes the sequential loop's decisions on its own vol
sums (fixed order), the oracle on correctly rounded sums; with the same
decisions the multiplier and the number of steps are bitwise equal, and with
eta = 0.5 or 1 (square root or nothing: correctly rounded operations only)
so are the updated densities and the change.  A decision may differ only
where vol at a midpoint lies within the rounding error of the device's sum
of V*: every test replays the device's path (rebuilt from its multiplier and
step count) and checks each decision against the oracle's correctly rounded
vol with that error bound, and one test puts V* exactly on such a tie."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import filters as OF
from oracle import oc as OC
from oracle import oracle as O
from paper_2505_02438_amd import api
from paper_2505_02438_amd import inputs as I

from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.01, 1.0, n)
    dc = -rng.exponential(2.0, n) * rho ** 2
    dc[:: 13] = 0.0                                    # B = 0: the lower move bound
    dv = rng.uniform(0.5, 1.5, n)
    return rho, dc, dv


def _check_decisions(rho, dc, dv, target, info, move, eta, tol, lmax=1e9, max_steps=200):
    """Replay the device's bisection path, recovered from its final multiplier
    and step count, and check every decision: vol(mid) > V* must send l1 to
    mid and vol(mid) < V* l2, with vol the oracle's correctly rounded sum,
    unless |vol(mid) - V*| is within the error bound of the device's
    fixed-order sum of n products (n u sum_e dv_e rho_new_e, u = 2^-53).
    Returns the number of decisions that fell within that bound."""
    lam_g, steps_g = info["lambda"], info["steps"]
    l1, l2 = 0.0, float(lmax)
    n, ties = len(rho), 0
    for k in range(steps_g):
        assert l2 - l1 > tol * (l1 + l2) and k < max_steps, "device ran more steps than the loop allows"
        mid = 0.5 * (l1 + l2)
        vol = OC.volume(dv, OC.oc_candidate(rho, dc, dv, mid, move, eta))
        bound = n * 2.0 ** -53 * vol
        if k == steps_g - 1:
            assert mid == lam_g, "the device's multiplier is not on its own path"
            break
        went_up = lam_g > mid               # the device set l1 = mid (it saw vol > V*)
        if abs(vol - target) > bound:
            assert went_up == (vol > target), f"step {k}: vol {vol!r} V* {target!r} decided the other way"
        else:
            ties += 1
        if went_up:
            l1 = mid
        else:
            l2 = mid
    else:
        assert steps_g == 0
    return ties


@pytest.mark.parametrize("n,eta,tol,move", [(5000, 0.5, 1e-3, 0.2), (5000, 1.0, 1e-3, 0.2), (5000, 0.5, 1e-12, 0.05),
                                            (777, 0.5, 1e-6, 1.0), (1, 0.5, 1e-3, 0.2), (256 * 1024 + 77, 0.5, 1e-4, 0.2)])
def test_oc_update_matches_oracle_bitwise(n, eta, tol, move):
    rho, dc, dv = _inputs(n, 41 + n)
    target = 0.4 * dv.sum()
    rn, lam, vol, steps, change = OC.oc_update(rho, dc, dv, target, move=move, eta=eta, tol=tol)
    got, info = api.oc_update(dev(rho), dev(dc), dev(dv), target, move=move, eta=eta, tol=tol)
    print(f"n={n} eta={eta} tol={tol}: steps {info['steps']} / {steps}, lambda {info['lambda']!r} / {lam!r}")
    ties = _check_decisions(rho, dc, dv, target, info, move, eta, tol)
    if ties == 0:
        # no decision within rounding: the paths, hence every result, agree
        assert info["steps"] == steps and info["lambda"] == lam
        assert np.array_equal(host(got), rn)
        assert info["change"] == change
        assert abs(info["volume"] - vol) <= 1e-13 * abs(vol)
    # whatever the path: the densities are the update at the device's multiplier
    assert np.array_equal(host(got), OC.oc_candidate(rho, dc, dv, info["lambda"], move, eta))


@pytest.mark.parametrize("tie_step", [3, 9, 17])
def test_oc_decisions_valid_at_a_tie(tie_step):
    """V* set exactly to the oracle's vol at the midpoint of one bisection
    step: there the oracle takes l2 = mid, and the device, whose sum may lie
    an ulp or so either side, may take either branch.  Every decision must be
    valid (above), and the densities are the update at the device's
    multiplier."""
    rho, dc, dv = _inputs(20000, 77 + tie_step)
    move, eta, tol = 0.2, 0.5, 1e-9
    l1, l2 = 0.0, 1e9
    target0 = 0.4 * dv.sum()
    for _ in range(tie_step):
        mid = 0.5 * (l1 + l2)
        v = OC.volume(dv, OC.oc_candidate(rho, dc, dv, mid, move, eta))
        if v > target0:
            l1 = mid
        else:
            l2 = mid
    mid = 0.5 * (l1 + l2)
    target = OC.volume(dv, OC.oc_candidate(rho, dc, dv, mid, move, eta))   # a tie at step tie_step
    got, info = api.oc_update(dev(rho), dev(dc), dev(dv), target, move=move, eta=eta, tol=tol)
    ties = _check_decisions(rho, dc, dv, target, info, move, eta, tol)
    print(f"tie at step {tie_step}: device steps {info['steps']}, decisions within rounding {ties}")
    assert ties >= 1
    assert np.array_equal(host(got), OC.oc_candidate(rho, dc, dv, info["lambda"], move, eta))


def test_oc_update_general_eta():
    """eta = 0.3 uses pow, whose last bit may differ between the two math
    libraries: the same decisions, densities within a few ulp."""
    rho, dc, dv = _inputs(20000, 42)
    target = 0.5 * dv.sum()
    rn, lam, vol, steps, change = OC.oc_update(rho, dc, dv, target, eta=0.3, tol=1e-6)
    got, info = api.oc_update(dev(rho), dev(dc), dev(dv), target, eta=0.3, tol=1e-6)
    assert info["steps"] == steps and info["lambda"] == lam
    np.testing.assert_allclose(host(got), rn, rtol=1e-14, atol=0)
    assert abs(info["change"] - change) <= 1e-14


def test_oc_update_limits_and_reuse():
    rho, dc, dv = _inputs(3000, 43)
    d_rho, d_dc, d_dv = dev(rho), dev(dc), dev(dv)
    # unreachable volumes: the step cap and the move limits decide
    for target, steps_cap in ((1e-9, 200), (1e9, 37)):
        rn, lam, vol, steps, change = OC.oc_update(rho, dc, dv, target, max_steps=steps_cap)
        got, info = api.oc_update(d_rho, d_dc, d_dv, target, max_steps=steps_cap)
        assert info["steps"] == steps and info["lambda"] == lam and np.array_equal(host(got), rn)
    # the workspace carries no state between calls: a second call of another size
    a, ia = api.oc_update(d_rho, d_dc, d_dv, 0.3 * dv.sum())
    b, ib = api.oc_update(d_rho[:100].contiguous(), d_dc[:100].contiguous(), d_dv[:100].contiguous(),
                          0.3 * dv[:100].sum())
    a2, ia2 = api.oc_update(d_rho, d_dc, d_dv, 0.3 * dv.sum())
    assert torch.equal(a, a2) and ia == ia2
    rn, lam, *_ = OC.oc_update(rho[:100], dc[:100], dv[:100], 0.3 * dv[:100].sum())
    assert ib["lambda"] == lam and np.array_equal(host(b), rn)


def _oracle_iteration(pr, rp, ci, H, rho, vf_target):
    m = pr.mesh
    K = O.assemble(m.elem, m.coords, m.cells, rho, rp, ci, pr.E0, pr.Emin, pr.p, pr.nu, pr.plane_strain, pr.mask)
    u = O.solve(rp, ci, K, pr.f)
    c = O.compliance(m.elem, m.coords, m.cells, rho, u, pr.f, pr.E0, pr.Emin, pr.p, pr.nu, pr.plane_strain)
    dc = O.sensitivity(m.elem, m.coords, m.cells, rho, u, pr.E0, pr.Emin, pr.p, pr.nu, pr.plane_strain)
    dcf = OF.sensitivity_filter(H, rho, dc)
    v = np.ones(len(rho))
    rn, lam, vol, steps, change = OC.oc_update(rho, dcf, v, vf_target, move=0.2, eta=0.5)
    return rn, c[1], lam, change


def test_optimisation_iterations_match_oracle():
    """Five iterations of Algorithm 1 on the 60 x 20 MBB half-beam (unit Q1,
    volume fraction 0.5, sensitivity filter r = 1.5, m = 0.2, eta = 0.5):
    GPU (assemble with Dirichlet, preconditioned CG to 1e-12, sensitivity, filter,
    OC) against the oracles (direct banded solve).  The compliances agree to
    the solver's accuracy and the densities closely: the bisection's
    decisions are the same."""
    pr = I.mbb_q1()
    m = pr.mesh
    n = m.n_cells
    rho0 = np.full(n, 0.5)
    target = 0.5 * n
    rp, ci = O.pattern(m.elem, m.n_nodes, m.cells)
    H = OF.filter_matrix(OF.centroids(m.elem, m.coords, m.cells), 1.5)
    pat = api.Pattern.from_mesh(m)
    flt = api.Filter.from_mesh(m, 1.5)
    mat = api.Material(E0=pr.E0, Emin=pr.Emin, nu=pr.nu, p=pr.p)
    mask, f, ones = dev(pr.mask), dev(pr.f), dev(np.ones(n))
    rho_g, rho_o = dev(rho0), rho0.copy()
    for it in range(5):
        K = pat.assemble(mat, rho_g, mask)
        u, iters, rel = pat.pcg(K, f, rtol=1e-12, max_iter=20000)
        dc, c = pat.evaluate(mat, rho_g, u, f=f)
        dcf = flt.sensitivity(rho_g, dc)
        rho_g, info = api.oc_update(rho_g, dcf, ones, target, move=0.2, eta=0.5)
        rho_o, c_o, lam_o, ch_o = _oracle_iteration(pr, rp, ci, H, rho_o, target)
        c_g = float(host(c)[1])
        print(f"iteration {it}: c {c_g:.10f} / {c_o:.10f}, lambda {info['lambda']:.6e} / {lam_o:.6e}, "
              f"change {info['change']:.4f}, CG {iters}")
        assert abs(c_g - c_o) <= 1e-9 * c_o
        assert abs(info["lambda"] - lam_o) <= 1e-9 * lam_o
        assert float(np.max(np.abs(host(rho_g) - rho_o))) <= 1e-8
    # the constraint holds and the design moved
    assert abs(float(host(rho_g).sum()) - target) <= 2e-3 * target


def test_density_filter_iterations_match_oracle():
    """Five iterations with the density filter (Sec. 2.4) instead: the
    physical density rho~ = F(rho) is assembled and evaluated, and the
    objective and volume sensitivities are taken back through the filter's
    chain rule (dv = F^T v, so the constraint is the filtered volume)."""
    pr = I.mbb_q1()
    m = pr.mesh
    n = m.n_cells
    target = 0.5 * n
    rp, ci = O.pattern(m.elem, m.n_nodes, m.cells)
    H = OF.filter_matrix(OF.centroids(m.elem, m.coords, m.cells), 2.5)
    v = np.ones(n)                                      # unit squares
    dv_o = OF.density_filter_backward(H, v, v)
    pat = api.Pattern.from_mesh(m)
    flt = api.Filter.from_mesh(m, 2.5)
    mat = api.Material(E0=pr.E0, Emin=pr.Emin, nu=pr.nu, p=pr.p)
    mask, f = dev(pr.mask), dev(pr.f)
    dv_g = flt.density_backward(dev(v))
    assert np.array_equal(host(dv_g), dv_o)
    rho_g, rho_o = dev(np.full(n, 0.5)), np.full(n, 0.5)
    for it in range(5):
        rt_g = flt.density(rho_g)
        K = pat.assemble(mat, rt_g, mask)
        u, iters, rel = pat.pcg(K, f, rtol=1e-12, max_iter=20000)
        dc, c = pat.evaluate(mat, rt_g, u, f=f)
        rho_g, info = api.oc_update(rho_g, flt.density_backward(dc), dv_g, target, move=0.2, eta=0.5)
        rt_o = OF.density_filter(H, v, rho_o)
        Ko = O.assemble(m.elem, m.coords, m.cells, rt_o, rp, ci, pr.E0, pr.Emin, pr.p, pr.nu, pr.plane_strain, pr.mask)
        uo = O.solve(rp, ci, Ko, pr.f)
        co = O.compliance(m.elem, m.coords, m.cells, rt_o, uo, pr.f, pr.E0, pr.Emin, pr.p, pr.nu, pr.plane_strain)[1]
        dco = O.sensitivity(m.elem, m.coords, m.cells, rt_o, uo, pr.E0, pr.Emin, pr.p, pr.nu, pr.plane_strain)
        rho_o, lam_o, *_ = OC.oc_update(rho_o, OF.density_filter_backward(H, v, dco), dv_o, target, move=0.2, eta=0.5)
        c_g = float(host(c)[1])
        print(f"density filter, iteration {it}: c {c_g:.10f} / {co:.10f}, lambda {info['lambda']:.6e} / {lam_o:.6e}")
        assert abs(c_g - co) <= 1e-9 * co
        assert abs(info["lambda"] - lam_o) <= 1e-9 * lam_o
        assert float(np.max(np.abs(host(rho_g) - rho_o))) <= 1e-8
    # the filtered volume meets the constraint
    assert abs(float(host(flt.density(rho_g)).sum()) - target) <= 2e-3 * target
