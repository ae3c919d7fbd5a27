"""Pins for the oracle's L-BFGS (the limited-memory variant the paper names as
the remedy for the O(d^2) update, Sec. VII): the two-loop recursion against
the inverse Hessian built explicitly by the rank-2 product form (Alg. 4's
update) from H0 = gamma I, and whole solves against closed-form minima."""
import numpy as np
import pytest

from paper_2603_28770_amd import workloads as W


def _dense_h(S, Y, d):
    """H after applying the product-form update for each pair, oldest first,
    starting from gamma I (gamma = s'y / y'y of the newest pair)."""
    sn, yn = S[-1], Y[-1]
    H = (sn @ yn) / (yn @ yn) * np.eye(d)
    for s, y in zip(S, Y):
        rho = 1.0 / (y @ s)
        A = np.eye(d) - rho * np.outer(s, y)
        H = A @ H @ A.T + rho * np.outer(s, s)
    return H


@pytest.mark.parametrize("d,m", [(1, 1), (3, 2), (10, 5), (40, 8)])
def test_two_loop_equals_explicit_inverse_hessian(oracle_any, d, m):
    rng = np.random.default_rng(d * 10 + m)
    Q = rng.standard_normal((d, d))
    A = Q @ Q.T + d * np.eye(d)          # SPD: y = A s gives y's > 0
    S = rng.standard_normal((m, d))
    Y = S @ A.T
    rho = 1.0 / np.einsum("ij,ij->i", Y, S)
    g = rng.standard_normal(d)
    p = oracle_any.lbfgs_direction(S, Y, rho, g)
    ref = -_dense_h(S, Y, d) @ g
    assert np.max(np.abs(p - ref)) <= 1e-11 * max(1.0, np.max(np.abs(ref)))


def test_two_loop_without_pairs_is_steepest_descent(oracle_any):
    g = np.array([1.5, -2.0, 0.25])
    p = oracle_any.lbfgs_direction(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), g)
    assert np.array_equal(p, -g)


def test_two_loop_one_pair_secant(oracle_any):
    """With one pair H y = s exactly in exact arithmetic (secant condition)."""
    rng = np.random.default_rng(3)
    s, y = rng.standard_normal(6), rng.standard_normal(6)
    if y @ s < 0:
        y = -y
    p = oracle_any.lbfgs_direction(s[None], y[None], np.array([1.0 / (y @ s)]), y)
    assert np.allclose(-p, s, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("obj,d", [("rosenbrock", 10), ("sphere", 30), ("quartic", 6)])
def test_lbfgs_solves_to_the_known_minimum(oracle_any, obj, d):
    lo, hi = (-2.0, 2.0)
    p = W.problem(objective=obj, dim=d, n=64, lower=lo, upper=hi, iter_pso=2, iter_bfgs=3000,
                  seed=4, lbfgs_m=6, grad_tol=1e-8)
    r = oracle_any.minimize(p)
    conv = r["status"] == 1
    assert conv.mean() >= 0.9
    fstar = W.f_star(obj, d)
    # the best start reaches the global minimum (quartic's is flat, f ~ |x|^4)
    assert r["f"][conv].min() - fstar <= (1e-10 if obj != "quartic" else 1e-6)
    # every converged start is a stationary point (Rosenbrock also has a local
    # minimum near x_1 = -1 for d >= 4)
    for i in np.flatnonzero(conv):
        _, g = oracle_any.grad(obj, r["x"][i])
        assert np.linalg.norm(g) < 1e-8


def test_lbfgs_differs_from_bfgs_only_in_the_direction(oracle_any):
    """m = 0 is BFGS; the swarm and first iterate do not depend on m."""
    p = W.problem(objective="rosenbrock", dim=5, n=32, lower=-2.0, upper=2.0, iter_pso=2,
                  iter_bfgs=200, seed=6)
    a = oracle_any.minimize(p)
    b = oracle_any.minimize(dict(p, lbfgs_m=4))
    assert np.array_equal(a["swarm"]["x"], b["swarm"]["x"])
    ta = oracle_any.bfgs(p, a["swarm"]["x"], trace_len=2)["trace"]
    tb = oracle_any.bfgs(dict(p, lbfgs_m=4), a["swarm"]["x"], trace_len=2)["trace"]
    assert np.array_equal(ta[:, :2], tb[:, :2])   # the first step is -g in both
