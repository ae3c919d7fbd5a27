"""Pins for the oracle's Armijo line search (Sec. III-D, Alg. 6) and rank-2
inverse-Hessian update (Sec. III-B, Alg. 4): worked examples whose every
value is exact in binary, the paper's product form of the update, the secant
condition, symmetry and positive definiteness."""
import numpy as np
import pytest

from paper_2603_28770_amd.workloads import problem


def _pb(obj, d, **kw):
    return problem(objective=obj, dim=d, n=1, lower=-1.0, upper=1.0, **kw)


@pytest.mark.parametrize("c", [1e-4, 0.3, 0.5])
def test_sphere_unit_step_accepted(oracle_any, c):
    # f = 0.5||x||^2, p = -g = -x: alpha = 1 lands on 0 and satisfies Armijo for c <= 1/2
    x = np.array([3.0, -4.0])
    a, trials, acc = oracle_any.line_search(_pb("sphere", 2, armijo_c=c), x, 12.5, -x, -25.0)
    assert (a, trials, acc) == (1.0, 1, True)


@pytest.mark.parametrize("d", [1, 3])
def test_quartic_backtracking_worked_example(oracle_any, d):
    # f = sum x^4 at x = 1: g = 4, p = -4, g'p = -16 d.  alpha = 1 -> f = 81 d and
    # alpha = 1/2 -> f = d are rejected; alpha = 1/4 -> f = 0 passes iff c <= 1/4.
    x, p, f0, ddir = np.ones(d), -4 * np.ones(d), float(d), -16.0 * d
    a, trials, acc = oracle_any.line_search(_pb("quartic", d, armijo_c=1e-4), x, f0, p, ddir)
    assert (a, trials, acc) == (0.25, 3, True)
    # the paper's c = 0.3 also rejects 1/4 (0 > d - 1.2 d is false... rhs < 0) and
    # accepts 1/8 -> x = 0.5, f = d/16 <= d - 0.6 d
    a, trials, acc = oracle_any.line_search(_pb("quartic", d, armijo_c=0.3), x, f0, p, ddir)
    assert (a, trials, acc) == (0.125, 4, True)


def test_line_search_exhausted_returns_shrunk_step(oracle_any):
    # no trial accepted within iter_ls: alpha has been shrunk iter_ls times
    x, p = np.ones(2), -4 * np.ones(2)
    a, trials, acc = oracle_any.line_search(_pb("quartic", 2, armijo_c=0.3, iter_ls=2), x, 2.0, p, -32.0)
    assert (a, trials, acc) == (0.25, 2, False)
    a, trials, acc = oracle_any.line_search(_pb("quartic", 2, armijo_c=0.3, iter_ls=1, ls_shrink=0.25),
                                            x, 2.0, p, -32.0)
    assert (a, trials, acc) == (0.25, 1, False)


def _spd(rng, d):
    A = rng.normal(size=(d, d))
    return A @ A.T + d * np.eye(d)


@pytest.mark.parametrize("d", [1, 2, 5, 16])
def test_update_equals_product_form(oracle_any, d):
    # H+ = (I - rho s y')H(I - rho y s') + rho s s', the form printed with Alg. 4
    rng = np.random.default_rng(d)
    for _ in range(10):
        H = _spd(rng, d)
        s, y = rng.normal(size=d), rng.normal(size=d)
        if s @ y <= 0:
            y = -y
        rho = 1.0 / (s @ y)
        I = np.eye(d)
        ref = (I - rho * np.outer(s, y)) @ H @ (I - rho * np.outer(y, s)) + rho * np.outer(s, s)
        Hn, applied = oracle_any.bfgs_update(H, s, y)
        assert applied
        assert np.max(np.abs(Hn - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("d", [2, 7, 32])
def test_update_secant_symmetry_definiteness(oracle_any, d):
    rng = np.random.default_rng(100 + d)
    for _ in range(10):
        H = _spd(rng, d)
        H = 0.5 * (H + H.T)
        s = rng.normal(size=d)
        y = _spd(rng, d) @ s                      # curvature pair of a convex quadratic
        Hn, applied = oracle_any.bfgs_update(H, s, y)
        assert applied
        err = np.linalg.norm(Hn @ y - s)
        assert err <= 1e-14 * d * np.linalg.norm(Hn) * np.linalg.norm(y)
        # symmetric up to the rounding of the fused row updates
        assert np.max(np.abs(Hn - Hn.T)) <= 8 * np.finfo(float).eps * np.max(np.abs(Hn))
        np.linalg.cholesky(Hn)                   # positive definite when y's > 0


def test_update_one_dimensional(oracle_any):
    Hn, applied = oracle_any.bfgs_update(np.array([[3.0]]), np.array([2.0]), np.array([0.5]))
    assert applied and abs(Hn[0, 0] - 4.0) <= 1e-14 * 4.0   # H+ = s / y


def test_update_skipped_without_curvature(oracle_any):
    H = np.eye(3)
    for y in (np.array([-1.0, 0.0, 0.0]), np.zeros(3)):
        Hn, applied = oracle_any.bfgs_update(H, np.array([1.0, 0.0, 0.0]), y)
        assert not applied and np.array_equal(Hn, H)
