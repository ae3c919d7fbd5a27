"""Whole-method pins for the oracle (Alg. 1 shape: PSO seeds, then BFGS from
every seed, then best-of-N): closed-form minima, brute-force grid search at
d = 2, the stationary points of separable objectives, the Ackley failure mode
of Sec. VI, the non-finite path, determinism and input validation."""
import math

import numpy as np
import pytest
import scipy.optimize as so

from paper_2603_28770_amd import workloads as W

CONV, MAXIT, NONF = 1, 0, 3


def test_rosenbrock_d2_config(oracle_any):
    r = oracle_any.minimize(W.ROSENBROCK_D2)
    assert r["best_f"] <= 1e-10
    assert np.max(np.abs(r["x"][r["best_index"]] - 1.0)) <= 1e-5
    assert r["n_converged"] >= 0.95 * W.ROSENBROCK_D2["n"]


def _grid_min(obj, lo, hi, n=2001):
    g = np.linspace(lo, hi, n)
    X, Y = np.meshgrid(g, g, indexing="ij")
    if obj == "rosenbrock":
        F = (1 - X) ** 2 + 100 * (Y - X * X) ** 2
    elif obj == "rastrigin":
        F = 20 + X * X - 10 * np.cos(2 * np.pi * X) + Y * Y - 10 * np.cos(2 * np.pi * Y)
    elif obj == "styblinski_tang":
        F = 0.5 * (X**4 - 16 * X**2 + 5 * X + Y**4 - 16 * Y**2 + 5 * Y)
    elif obj == "goldstein_price":
        F = ((1 + (X + Y + 1) ** 2 * (19 - 14 * X + 3 * X * X - 14 * Y + 6 * X * Y + 3 * Y * Y))
             * (30 + (2 * X - 3 * Y) ** 2 * (18 - 32 * X + 12 * X * X + 48 * Y - 36 * X * Y + 27 * Y * Y)))
    k = np.unravel_index(np.argmin(F), F.shape)
    return np.array([g[k[0]], g[k[1]]])


@pytest.mark.parametrize("obj,lo,hi", [("rosenbrock", -5.0, 5.0), ("rastrigin", -5.12, 5.12),
                                       ("styblinski_tang", -5.0, 5.0), ("goldstein_price", -2.0, 2.0)])
def test_brute_force_grid_d2(oracle_any, obj, lo, hi):
    x0 = _grid_min(obj, lo, hi)
    # polish the grid point with scipy's own BFGS on the oracle's values
    res = so.minimize(lambda x: oracle_any.f(obj, x), x0, method="Nelder-Mead",
                      options=dict(xatol=1e-12, fatol=1e-15, maxiter=20000))
    p = W.problem(objective=obj, dim=2, n=512, lower=lo, upper=hi, iter_pso=5, iter_bfgs=500,
                  seed=17)
    r = oracle_any.minimize(p)
    assert abs(r["best_f"] - res.fun) <= 1e-8 * max(1.0, abs(res.fun))
    assert abs(r["best_f"] - W.f_star(obj, 2)) <= 1e-8 * max(1.0, abs(W.f_star(obj, 2)))


def test_ackley_grid_d2(oracle_any):
    # the grid contains the origin; BFGS reaches it only up to the cone's kink
    p = W.problem(objective="ackley", dim=2, n=512, lower=-5.0, upper=5.0, iter_pso=5,
                  iter_bfgs=500, seed=17)
    r = oracle_any.minimize(p)
    assert r["best_f"] <= 1e-8


def _rastrigin_stationary_1d():
    # roots of d/dx [x^2 - 10 cos(2 pi x)] = 2x + 20 pi sin(2 pi x); none beyond |x| = 10 pi
    h = lambda x: 2 * x + 20 * math.pi * math.sin(2 * math.pi * x)
    grid = np.linspace(-33, 33, 132001)
    vals = [h(x) for x in grid]
    roots = [0.0]
    for a, b, fa, fb in zip(grid[:-1], grid[1:], vals[:-1], vals[1:]):
        if fa == 0.0 or fa * fb < 0:
            r = so.brentq(h, a, b, xtol=1e-15) if fa != 0.0 else a
            if abs(r) > 1e-12:
                roots.append(r)
    return np.array(sorted(roots))


def test_rastrigin_endpoints_are_stationary_points(oracle_any):
    roots = _rastrigin_stationary_1d()
    assert np.min(np.abs(roots - 0.994958637652335)) < 1e-12
    p = W.problem(objective="rastrigin", dim=6, n=512, lower=-5.12, upper=5.12, iter_pso=3,
                  iter_bfgs=1000, seed=3)
    r = oracle_any.minimize(p)
    conv = r["status"] == CONV
    assert conv.mean() > 0.9
    # ||g|| < 1e-6 puts every coordinate within ~2.5e-9 of a 1-D stationary point
    dist = np.min(np.abs(r["x"][conv][:, :, None] - roots[None, None, :]), axis=2)
    assert dist.max() < 1e-8
    assert np.all(r["f"][conv] >= -1e-12)


def test_styblinski_tang_endpoints(oracle_any):
    stationary = np.array([W.ST_XSTAR, 0.15673157, 2.746802770990838])  # roots of 4x^3 - 32x + 5
    assert np.allclose(np.sort(np.roots([4, 0, -32, 5]).real), stationary, atol=1e-7)
    p = W.problem(objective="styblinski_tang", dim=8, n=256, lower=-5.0, upper=5.0, iter_pso=2,
                  iter_bfgs=500, seed=8)
    r = oracle_any.minimize(p)
    conv = r["status"] == CONV
    assert conv.mean() > 0.9
    dist = np.min(np.abs(r["x"][conv][:, :, None] - stationary[None, None, :]), axis=2)
    assert dist.max() < 1e-7
    assert r["best_f"] >= W.ST_FSTAR_PER_DIM * 8 - 1e-9


@pytest.mark.parametrize("d", [2, 5])
def test_ackley_failure_mode_near_origin(oracle_any, d):
    # Sec. VI: near the kink at 0 the gradient norm stays near the cone slope
    # 4/sqrt(d), so the ||g|| < Theta test never fires and the starts run out
    # of iterations while hopping around the minimum
    p = W.problem(objective="ackley", dim=d, n=64, lower=-0.1, upper=0.1, iter_bfgs=200, seed=5)
    r = oracle_any.minimize(p)
    near = np.max(np.abs(r["x"]), axis=1) < 1e-3
    assert near.mean() >= 0.8
    assert np.all(r["status"][near] == MAXIT) and np.all(r["iters"][near] == 200)
    # the cone: f ~ 4 ||x|| / sqrt(d) next to the origin
    rn = np.linalg.norm(r["x"][near], axis=1)
    assert np.all(r["f"][near] <= 5 * rn / math.sqrt(d) + 1e-14)
    for x in r["x"][near]:
        _, g = oracle_any.grad("ackley", x)
        # cone slope plus the O(||x||) pull of the cosine term (2 pi)^2 e x / d
        assert abs(np.linalg.norm(g) - 4 / math.sqrt(d)) < 1e-6 + 120 * np.linalg.norm(x) / d


def test_non_finite_start(oracle_any):
    p = W.problem(objective="rosenbrock", dim=3, n=8, lower=1e200, upper=2e200, iter_bfgs=10)
    r = oracle_any.minimize(p)
    assert np.all(r["status"] == NONF) and np.all(r["iters"] == 0)
    assert r["best_index"] == -1 and r["n_converged"] == 0


def test_zero_bfgs_budget_returns_seeds(oracle_any):
    p = W.problem(objective="rastrigin", dim=4, n=32, lower=-5.12, upper=5.12, iter_pso=2,
                  iter_bfgs=0, seed=1)
    r = oracle_any.minimize(p)
    sw = r["swarm"]
    assert np.array_equal(r["x"], sw["x"]) and np.all(r["iters"] == 0)
    assert np.all(r["status"] == MAXIT)
    assert all(r["f"][i] == oracle_any.f("rastrigin", sw["x"][i]) for i in range(32))


def test_sphere_converges_in_one_exact_step(oracle_any):
    p = W.problem(objective="sphere", dim=5, n=64, lower=-3.0, upper=3.0, iter_pso=2, seed=2)
    r = oracle_any.minimize(p)
    assert np.all(r["status"] == CONV) and np.all(r["iters"] == 1) and np.all(r["x"] == 0.0)


def test_quartic_worked_first_step(oracle_any):
    p = W.problem(objective="quartic", dim=3, n=1, lower=-1.0, upper=1.0, armijo_c=1e-4)
    r = oracle_any.bfgs(p, np.ones((1, 3)), trace_len=3)
    # alpha = 1/4 lands on the minimum exactly and the gradient there is 0
    assert r["status"][0] == CONV and r["iters"][0] == 1 and np.all(r["x"][0] == 0.0)
    assert r["ls_trials"][0] == 3
    assert np.array_equal(r["trace"][0, 0], np.ones(3)) and np.all(r["trace"][0, 1] == 0.0)


def test_deterministic_and_thread_invariant(oracle_any):
    p = W.scaled(W.RASTRIGIN_D10, 256)
    a = oracle_any.minimize(p, nthreads=1)
    b = oracle_any.minimize(p, nthreads=4)
    for k in ("x", "f", "iters", "status", "ls_trials"):
        assert np.array_equal(a[k], b[k])


@pytest.mark.parametrize("bad", [dict(dim=0), dict(n=0), dict(lower=1.0, upper=1.0),
                                 dict(upper=float("inf")), dict(iter_ls=0), dict(iter_bfgs=-1),
                                 dict(iter_pso=-1), dict(grad_tol=0.0), dict(armijo_c=1.0),
                                 dict(ls_shrink=0.0), dict(w=float("nan")),
                                 dict(objective="rosenbrock", dim=1),
                                 dict(objective="goldstein_price", dim=3)])
def test_validation(oracle_any, bad):
    p = W.problem(objective="sphere", dim=2, n=4, lower=-1.0, upper=1.0)
    assert oracle_any.validate(p)
    p.update(bad)
    assert not oracle_any.validate(p)
