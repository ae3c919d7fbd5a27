"""Pins for the oracle's sin, cos and exp: in the default build Cody-Waite
reduction + Taylor series with fused multiply-adds, which the objectives
evaluate instead of the C library; in the plain build the C library's.  Both
are held to the same bars: error against an extended-precision reference,
exact special values and symmetries, large arguments up to 2^48; beyond that
the default build's sin and cos are NaN."""
import ctypes as C

import numpy as np
import pytest


@pytest.fixture(scope="module")
def M(oracle_any):
    L = oracle_any.lib()
    for n in ("zo_sin", "zo_cos", "zo_exp"):
        getattr(L, n).restype = C.c_double
        getattr(L, n).argtypes = [C.c_double]
    L.plain = oracle_any.plain
    return L


def _ulps(vals, ref_ld):
    ref = ref_ld.astype(np.float64)   # correctly rounded to double (80-bit reference)
    err = np.abs(vals - ref) / np.spacing(np.abs(ref))
    return float(np.max(err))


@pytest.mark.parametrize("lo,hi", [(-1.0, 1.0), (-40.0, 40.0), (-3.3e4, 3.3e4), (-1e8, 1e8)])
def test_sin_cos_within_one_ulp(M, lo, hi):
    x = np.random.default_rng(int(hi)).uniform(lo, hi, 20000)
    xl = x.astype(np.longdouble)
    s = np.array([M.zo_sin(v) for v in x])
    c = np.array([M.zo_cos(v) for v in x])
    assert _ulps(s, np.sin(xl)) <= 1.0
    assert _ulps(c, np.cos(xl)) <= 1.0


def test_sin_cos_near_multiples_of_half_pi(M):
    # arguments 2 pi x for x next to the Rastrigin minima, where the reduced
    # argument cancels almost completely
    k = np.arange(-20, 21)
    x = np.concatenate([k * 0.5 + d for d in (1e-12, -3e-9, 2e-6, 0.0)])
    t = 6.283185307179586 * x
    tl = t.astype(np.longdouble)
    assert _ulps(np.array([M.zo_sin(v) for v in t]), np.sin(tl)) <= 1.0
    assert _ulps(np.array([M.zo_cos(v) for v in t]), np.cos(tl)) <= 1.0


def test_exp_within_one_ulp(M):
    x = np.concatenate([np.random.default_rng(3).uniform(-700, 700, 20000),
                        np.random.default_rng(4).uniform(-1, 1, 5000)])
    e = np.array([M.zo_exp(v) for v in x])
    assert _ulps(e, np.exp(x.astype(np.longdouble))) <= 1.0


def test_special_values(M):
    assert M.zo_sin(0.0) == 0.0 and M.zo_cos(0.0) == 1.0 and M.zo_exp(0.0) == 1.0
    assert M.zo_exp(1.0) == np.e or abs(M.zo_exp(1.0) - np.e) <= np.spacing(np.e)
    assert M.zo_exp(1000.0) == np.inf and M.zo_exp(-1000.0) == 0.0
    assert M.zo_exp(-np.inf) == 0.0 and M.zo_exp(np.inf) == np.inf
    with np.errstate(invalid="ignore"):
        assert np.isnan(M.zo_exp(np.nan)) and np.isnan(M.zo_cos(np.inf))
        assert np.isnan(M.zo_sin(np.nan))
    # subnormal results still follow exp
    v = M.zo_exp(-740.0)
    assert 0.0 < v < 1e-300 and abs(v - np.exp(np.longdouble(-740.0))) <= 2 * np.spacing(v)


def test_symmetries(M):
    x = np.random.default_rng(5).uniform(-100, 100, 2000)
    for v in x:
        assert M.zo_sin(-v) == -M.zo_sin(v) and M.zo_cos(-v) == M.zo_cos(v)


@pytest.mark.parametrize("lo,hi", [(2.0 ** 28, 2.0 ** 38), (2.0 ** 38, 2.0 ** 47.99)])
def test_large_arguments_keep_the_reduction_accurate(M, lo, hi):
    # the fused three-part reduction stays accurate while rint(x 2/pi) is the
    # nearest integer: absolute error within an ulp of 1 against 80-bit sin/cos
    rng = np.random.default_rng(int(np.log2(lo)))
    x = np.exp(rng.uniform(np.log(lo), np.log(hi), 5000)) * rng.choice([-1.0, 1.0], 5000)
    xl = x.astype(np.longdouble)
    s = np.array([M.zo_sin(v) for v in x])
    c = np.array([M.zo_cos(v) for v in x])
    assert np.max(np.abs(s - np.sin(xl).astype(np.float64))) <= np.spacing(1.0)
    assert np.max(np.abs(c - np.cos(xl).astype(np.float64))) <= np.spacing(1.0)


def test_out_of_range_arguments_are_nan(M):
    if M.plain:
        pytest.skip("the C library reduces every finite argument")
    for v in (2.0 ** 48, -(2.0 ** 48), 1e300, np.inf, -np.inf, np.nan):
        assert np.isnan(M.zo_sin(v)) and np.isnan(M.zo_cos(v))
    v = np.nextafter(2.0 ** 48, 0.0)
    assert abs(M.zo_sin(v) - float(np.sin(np.longdouble(v)))) <= np.spacing(1.0)
