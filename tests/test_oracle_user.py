"""Pins for the oracle's user-objective path and its logarithm.

* zo_log (reduction to [sqrt(1/2), sqrt(2)) and the atanh series): error
  against an extended-precision reference, exact and special values.
* A user objective compiled for the CPU against the oracle's dual numbers:
  user sources that restate built-in test functions give the built-in
  oracle's values and gradients (same operation sequence), closed forms,
  scipy's Rosenbrock derivative, exact integer cases, finite differences for a
  Poisson likelihood, and a whole BFGS solve of Goldstein-Price reaching its
  known minimum 3 at (0, -1)."""
import ctypes as C

import numpy as np
import pytest

from oracle import user as U
from paper_2603_28770_amd import user_objectives as UO
from paper_2603_28770_amd import workloads as W


@pytest.fixture(scope="module")
def L(oracle_mod):
    L = oracle_mod.lib()
    L.zo_log.restype = C.c_double
    L.zo_log.argtypes = [C.c_double]
    return L


def _ulps(vals, ref_ld):
    ref = ref_ld.astype(np.float64)
    return float(np.max(np.abs(vals - ref) / np.spacing(np.abs(ref))))


@pytest.mark.parametrize("lo,hi", [(0.5, 2.0), (1e-3, 1e3), (1e-300, 1e300)])
def test_log_within_two_ulp(L, lo, hi):
    x = np.exp(np.random.default_rng(int(np.log10(hi)) + 7).uniform(np.log(lo), np.log(hi), 20000))
    got = np.array([L.zo_log(v) for v in x])
    ref = np.log(x.astype(np.longdouble))
    keep = np.abs(ref) > 1e-3  # relative error is measured away from log = 0
    assert _ulps(got[keep], ref[keep]) <= 2.0


def test_log_exact_and_special(L):
    assert L.zo_log(1.0) == 0.0
    for k in (-1074, -1022, -3, 1, 2, 10, 1023):
        ref = np.longdouble(k) * np.log(np.longdouble(2))
        assert abs(L.zo_log(2.0 ** k) - float(ref)) <= np.spacing(abs(float(ref)))
    # near 1 (the reference is log1p of the exact difference x - 1)
    for h in (2.0 ** -30, -(2.0 ** -30), 1e-12, -3e-9):
        x = 1.0 + h
        ref = np.log1p(np.longdouble(x) - np.longdouble(1.0))
        assert abs(L.zo_log(x) - float(ref)) <= 2 * np.spacing(abs(float(ref)))
    assert L.zo_log(0.0) == -np.inf and L.zo_log(np.inf) == np.inf
    assert np.isnan(L.zo_log(-1.0)) and np.isnan(L.zo_log(np.nan))


def _val_grad(oracle_mod, src, x):
    U.use(src, oracle_mod.lib())
    f = oracle_mod.f("user", np.asarray(x, dtype=np.float64))
    fv, g = oracle_mod.grad("user", np.asarray(x, dtype=np.float64))
    assert fv == f
    return f, g


def test_user_restatements_equal_builtins(oracle_mod):
    rng = np.random.default_rng(3)
    for _ in range(20):
        x = rng.uniform(-2, 2, 2)
        f, g = _val_grad(oracle_mod, UO.ROSENBROCK, x)  # d = 2: one term, no sum order
        assert f == oracle_mod.f("rosenbrock", x)
        assert np.array_equal(g, oracle_mod.grad("rosenbrock", x)[1])
        f, g = _val_grad(oracle_mod, UO.GOLDSTEIN_PRICE, x)
        assert f == oracle_mod.f("goldstein_price", x)
        assert np.array_equal(g, oracle_mod.grad("goldstein_price", x)[1])


def test_user_closed_forms(oracle_mod):
    import scipy.optimize as so
    f, g = _val_grad(oracle_mod, UO.ROSENBROCK, [-1.2, 1.0])
    assert abs(f - 24.2) < 1e-14 and np.allclose(g, [-215.6, -88.0], rtol=1e-14, atol=0)
    x = np.random.default_rng(5).uniform(-2, 2, 7)
    f, g = _val_grad(oracle_mod, UO.ROSENBROCK, x)
    assert np.allclose(g, so.rosen_der(x), rtol=1e-13, atol=1e-13)
    f, g = _val_grad(oracle_mod, UO.GOLDSTEIN_PRICE, [0.0, -1.0])
    assert f == 3.0 and np.array_equal(g, [0.0, 0.0])


def test_user_integer_sum_of_squares_is_exact(oracle_mod):
    src = '''
template <class T, class X>
ZEUS_FN T objective(const X &x, int d) {
  T s = T(0.0);
  for (int i = 0; i < d; ++i) s = s + x[i] * x[i];
  return s;
}
'''
    x = np.arange(-5, 6, dtype=np.float64)
    f, g = _val_grad(oracle_mod, src, x)
    assert f == float(np.sum(x * x)) and np.array_equal(g, 2 * x)


def test_user_poisson_likelihood_gradient(oracle_mod):
    src = UO.poisson_fit_source(UO.POISSON_COUNTS)
    theta = np.array(UO.POISSON_TRUE) * np.array([1.1, 0.9, 1.05, 0.8])
    f, g = _val_grad(oracle_mod, src, theta)
    assert np.isfinite(f)
    for j in range(theta.size):
        h = 1e-6 * max(1.0, abs(theta[j]))
        e = np.zeros_like(theta)
        e[j] = h
        fd = (oracle_mod.f("user", theta + e) - oracle_mod.f("user", theta - e)) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j]))


def test_user_bfgs_finds_goldstein_price_minimum(oracle_mod):
    U.use(UO.GOLDSTEIN_PRICE, oracle_mod.lib())
    p = W.problem(objective="user", dim=2, n=256, lower=-2.0, upper=2.0, iter_pso=5, iter_bfgs=200,
                  seed=4)
    out = oracle_mod.minimize(p)
    best = int(np.argmin(np.where(np.isfinite(out["f"]), out["f"], np.inf)))
    assert abs(out["f"][best] - 3.0) < 1e-10
    assert np.allclose(out["x"][best], [0.0, -1.0], atol=1e-6)
