"""Pins of the OC oracle (Sec. 2.3, Algorithm 1) against facts other than
itself: the three cases of the update worked by hand, a closed-form
multiplier for identical elements, the root of vol(lambda) = V* found by an
independent root finder (scipy's brentq), monotonicity of vol, and the move
limit's extremes."""
import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import oc as OC


def test_update_cases_by_hand():
    rho = np.array([0.5, 0.5, 0.5, 0.05, 0.95])
    dc = np.array([-1.0, -100.0, -0.01, -0.0001, -1e6])
    dv = np.ones(5)
    got = OC.oc_candidate(rho, dc, dv, lam=1.0, move=0.2, eta=0.5)
    # 0.5 sqrt(1) = 0.5 inside; 0.5 * 10 = 5 -> min(1, 0.7) = 0.7; 0.5 * 0.1 = 0.05 -> max(0, 0.3) = 0.3;
    # 0.05 * 0.01 = 5e-4 -> max(0, -0.15) = 0 wins over ... 5e-4 is above 0, inside; 0.95 * 1000 -> min(1, 1.15) = 1
    np.testing.assert_array_equal(got, [0.5, 0.7, 0.3, 0.05 * 0.01, 1.0])
    # eta = 1 and a general eta
    np.testing.assert_allclose(OC.oc_candidate([0.5], [-1.21], [1.0], 1.0, 0.5, 1.0), [0.5 * 1.21], rtol=1e-15)
    np.testing.assert_allclose(OC.oc_candidate([0.5], [-1.21], [2.0], 1.1, 0.5, 0.3),
                               [0.5 * (1.21 / 2.2) ** 0.3], rtol=1e-15)
    # a positive dc gives B = 0: the lower move bound
    assert OC.oc_candidate([0.5], [3.0], [1.0], 1.0, 0.2, 0.5)[0] == 0.3


def test_identical_elements_closed_form():
    """rho = 0.5, dc = -4, dv = 1: rho_new = 0.5 sqrt(4 / lambda) = lambda^-1/2; V* = 0.4 n
    needs rho_new = 0.4, so lambda* = 6.25 (inside the move limits 0.3 .. 0.7)."""
    n = 1000
    rn, lam, vol, steps, change = OC.oc_update(np.full(n, 0.5), np.full(n, -4.0), np.ones(n), 0.4 * n,
                                               move=0.2, eta=0.5, tol=1e-10)
    assert abs(lam - 6.25) <= 1e-9 * 6.25
    np.testing.assert_allclose(rn, 0.4, rtol=1e-9)
    assert abs(change - 0.1) <= 1e-9 and abs(vol - 400.0) <= 1e-6
    # the number of halvings from [0, 1e9] to a relative bracket of 1e-10
    assert 60 <= steps <= 75


@pytest.mark.parametrize("seed,eta", [(1, 0.5), (2, 1.0), (3, 0.3)])
def test_lambda_is_the_root_of_the_volume_constraint(seed, eta):
    rng = np.random.default_rng(seed)
    n = 5000
    rho = rng.uniform(0.01, 1.0, n)
    dc = -rng.exponential(2.0, n) * rho ** 2
    dv = rng.uniform(0.5, 1.5, n)
    target = 0.45 * dv.sum()
    tol = 1e-6
    rn, lam, vol, steps, change = OC.oc_update(rho, dc, dv, target, move=0.2, eta=eta, tol=tol)

    def f(lmb):
        return OC.volume(dv, OC.oc_candidate(rho, dc, dv, lmb, 0.2, eta)) - target

    root = brentq(f, 1e-12, 1e9, xtol=1e-300, rtol=1e-15)
    assert abs(lam - root) <= 2 * tol * root
    assert abs(vol - target) <= 1e-3 * target
    np.testing.assert_array_equal(rn, OC.oc_candidate(rho, dc, dv, lam, 0.2, eta))
    assert change == float(np.max(np.abs(rn - rho)))
    # vol is non-increasing in lambda
    grid = np.geomspace(root / 100, root * 100, 60)
    vols = [f(g) for g in grid]
    assert all(a >= b for a, b in zip(vols, vols[1:]))


def test_move_limit_extremes():
    rng = np.random.default_rng(4)
    n = 300
    rho = rng.uniform(0.3, 0.9, n)
    dc = -rng.uniform(0.5, 2.0, n)
    dv = np.ones(n)
    # unreachable small volume: every element moves down by m
    rn, lam, vol, steps, change = OC.oc_update(rho, dc, dv, 1e-6, move=0.1, eta=0.5)
    np.testing.assert_array_equal(rn, np.maximum(0.0, rho - 0.1))
    assert abs(change - 0.1) < 1e-15 and lam > 1e8
    # unreachable large volume: every element moves up by m (capped at 1)
    rn, lam, vol, steps, change = OC.oc_update(rho, dc, dv, 10.0 * n, move=0.1, eta=0.5, max_steps=400)
    np.testing.assert_array_equal(rn, np.minimum(1.0, rho + 0.1))
    # the step cap stops the loop
    *_, steps, _ = OC.oc_update(rho, dc, dv, 0.5 * n, tol=1e-15, max_steps=17)
    assert steps == 17
