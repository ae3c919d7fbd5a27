"""Pins for the oracle's objectives (Sec. V-B) and its forward-mode dual-number
gradient (Sec. III-C, Alg. 5): closed forms, an independent library, an
independent forward-mode AD, analytic derivatives and finite differences."""
import math

import numpy as np
import pytest
import scipy.optimize as so

from paper_2603_28770_amd.workloads import ST_FSTAR_PER_DIM, ST_XSTAR

DIMS = [2, 3, 7, 10, 50]
OBJ = ["rosenbrock", "rastrigin", "ackley", "styblinski_tang", "sphere", "quartic"]


# ---- values -----------------------------------------------------------------

@pytest.mark.parametrize("d", DIMS)
def test_minima_closed_forms(oracle_any, d):
    O = oracle_any
    assert O.f("rosenbrock", np.ones(d)) == 0.0
    assert O.f("rastrigin", np.zeros(d)) == 0.0
    assert abs(O.f("ackley", np.zeros(d))) <= 4.5e-16
    assert abs(O.f("styblinski_tang", np.full(d, ST_XSTAR)) - ST_FSTAR_PER_DIM * d) <= 1e-12 * d
    assert O.f("sphere", np.zeros(d)) == 0.0 and O.f("quartic", np.zeros(d)) == 0.0


def test_term_sums_are_balanced_pairwise(oracle_mod):
    """The paper leaves the order of the sum over terms open; the oracle adds
    pairwise (first h terms + the rest, h the largest power of two below the
    count).  Worked by hand with squares 2^54 (x = 2^27) and ones, where
    ulp(2^54) = 4 and 2^54 + 2 is a tie that rounds to even (2^54):
      d=8, x = (2^27, 1 x7): ((2^54+1)+(1+1)) + ((1+1)+(1+1)) = 2^54 + 4,
           so 0.5 sum = 2^53 + 2 (left to right: every +1 is lost, 2^53);
      d=7, x = (1 x6, 2^27): (1+1+1+1) + ((1+1) + 2^54) = 2^54 + 4, so
           2^53 + 2 (left to right: 6 + 2^54 rounds to 2^54 + 8, 2^53 + 4)."""
    O = oracle_mod
    assert O.f("sphere", [2.0 ** 27] + [1.0] * 7) == 2.0 ** 53 + 2
    assert O.f("sphere", [1.0] * 6 + [2.0 ** 27]) == 2.0 ** 53 + 2
    # the same sums through the dual-number path (value part of the gradient pass)
    f, _ = O.grad("sphere", [2.0 ** 27] + [1.0] * 7)
    assert f == 2.0 ** 53 + 2


def test_term_sums_left_to_right_in_the_plain_build():
    """The plain build adds an objective's terms strictly left to right.  The
    same hand-worked sums as above (ulp(2^54) = 4, ties to even):
      d=8, x = (2^27, 1 x7): 2^54 + 1 rounds to 2^54 and so does every later
           + 1, so 0.5 sum = 2^53;
      d=7, x = (1 x6, 2^27): 6 + 2^54 is a tie between 2^54 + 4 and
           2^54 + 8 and rounds to the even 2^54 + 8, so 0.5 sum = 2^53 + 4."""
    from oracle import oracle as O
    assert O.f("sphere", [2.0 ** 27] + [1.0] * 7, plain=True) == 2.0 ** 53
    assert O.f("sphere", [1.0] * 6 + [2.0 ** 27], plain=True) == 2.0 ** 53 + 4
    f, _ = O.grad("sphere", [1.0] * 6 + [2.0 ** 27], plain=True)
    assert f == 2.0 ** 53 + 4


def test_goldstein_price_values(oracle_any):
    assert oracle_any.f("goldstein_price", [0.0, -1.0]) == 3.0
    # by hand: A = 1 + 3^2 * 3 = 28, B = 30 + (-1)^2 * 37 = 67
    assert oracle_any.f("goldstein_price", [1.0, 1.0]) == 28.0 * 67.0


def test_rosenbrock_worked_value_and_scipy(oracle_any):
    assert abs(oracle_any.f("rosenbrock", [-1.2, 1.0]) - 24.2) <= 1e-14 * 24.2
    rng = np.random.default_rng(0)
    for d in DIMS:
        for _ in range(20):
            x = rng.uniform(-5, 5, d)
            ref = so.rosen(x)
            assert abs(oracle_any.f("rosenbrock", x) - ref) <= 1e-13 * max(1.0, abs(ref))


@pytest.mark.parametrize("d", [1, 2, 10])
def test_rastrigin_on_lattice(oracle_any, d):
    # integer points: cos(2 pi k) = 1 -> f = sum k^2; half-integers: cos = -1
    rng = np.random.default_rng(d)
    for _ in range(20):
        k = rng.integers(-5, 6, d).astype(float)
        assert abs(oracle_any.f("rastrigin", k) - np.sum(k * k)) <= 1e-11
        h = k + 0.5
        assert abs(oracle_any.f("rastrigin", h) - (20.0 * d + np.sum(h * h))) <= 1e-11


@pytest.mark.parametrize("d", [2, 5, 50])
def test_ackley_on_lattice(oracle_any, d):
    # x on the integer lattice: the cosine mean is exactly 1, so
    # f = 20 - 20 exp(-0.2 sqrt(mean x^2))
    rng = np.random.default_rng(d)
    for _ in range(20):
        k = rng.integers(-4, 5, d).astype(float)
        ref = 20.0 - 20.0 * math.exp(-0.2 * math.sqrt(np.mean(k * k)))
        assert abs(oracle_any.f("ackley", k) - ref) <= 1e-13


def test_styblinski_tang_values(oracle_any):
    for d in (1, 4, 9):
        assert oracle_any.f("styblinski_tang", np.zeros(d)) == 0.0
        assert oracle_any.f("styblinski_tang", np.ones(d)) == -5.0 * d
        assert oracle_any.f("styblinski_tang", np.full(d, 2.0)) == 0.5 * (16 - 64 + 10) * d


# ---- gradients ----------------------------------------------------------------

def _analytic(obj, x):
    d = x.size
    if obj == "rastrigin":
        return 2 * x + 20 * np.pi * np.sin(2 * np.pi * x)
    if obj == "styblinski_tang":
        return 2 * x**3 - 16 * x + 2.5
    if obj == "sphere":
        return x.copy()
    if obj == "quartic":
        return 4 * x**3
    if obj == "ackley":
        r = np.sqrt(np.sum(x * x) / d)
        e1 = np.exp(-0.2 * r)
        e2 = np.exp(np.sum(np.cos(2 * np.pi * x)) / d)
        return 4.0 * e1 * x / (d * r) + (2 * np.pi / d) * e2 * np.sin(2 * np.pi * x)
    raise KeyError(obj)


def test_rosenbrock_gradient_worked_and_scipy(oracle_any):
    f, g = oracle_any.grad("rosenbrock", [-1.2, 1.0])
    assert np.allclose(g, [-215.6, -88.0], rtol=1e-14, atol=0)
    rng = np.random.default_rng(1)
    for d in DIMS:
        for _ in range(10):
            x = rng.uniform(-5, 5, d)
            f, g = oracle_any.grad("rosenbrock", x)
            ref = so.rosen_der(x)
            assert np.max(np.abs(g - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
            assert f == oracle_any.f("rosenbrock", x)   # value part == primal


@pytest.mark.parametrize("obj", ["rastrigin", "styblinski_tang", "sphere", "quartic", "ackley"])
@pytest.mark.parametrize("d", [1, 2, 10, 50])
def test_gradient_vs_analytic(oracle_any, obj, d):
    rng = np.random.default_rng(d)
    for _ in range(10):
        x = rng.uniform(-5, 5, d)
        f, g = oracle_any.grad(obj, x)
        ref = _analytic(obj, x)
        assert np.max(np.abs(g - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref))), (obj, d)
        assert f == oracle_any.f(obj, x)


def _torch_obj(obj):
    import torch

    def rosen(x):
        return torch.sum((1 - x[:-1]) ** 2 + 100 * (x[1:] - x[:-1] ** 2) ** 2)

    def rast(x):
        return 10 * x.numel() + torch.sum(x * x - 10 * torch.cos(2 * math.pi * x))

    def ackley(x):
        d = x.numel()
        return (-20 * torch.exp(-0.2 * torch.sqrt(torch.sum(x * x) / d))
                - torch.exp(torch.sum(torch.cos(2 * math.pi * x)) / d) + 20 + math.e)

    def st(x):
        return 0.5 * torch.sum(x**4 - 16 * x**2 + 5 * x)

    def gp(x):
        a, b = x[0], x[1]
        A = 1 + (a + b + 1) ** 2 * (19 - 14 * a + 3 * a * a - 14 * b + 6 * a * b + 3 * b * b)
        B = 30 + (2 * a - 3 * b) ** 2 * (18 - 32 * a + 12 * a * a + 48 * b - 36 * a * b + 27 * b * b)
        return A * B
    return {"rosenbrock": rosen, "rastrigin": rast, "ackley": ackley, "styblinski_tang": st,
            "goldstein_price": gp}[obj]


@pytest.mark.parametrize("obj", ["rosenbrock", "rastrigin", "ackley", "styblinski_tang",
                                 "goldstein_price"])
def test_gradient_vs_torch_forward_mode(oracle_any, obj):
    torch = pytest.importorskip("torch")
    from torch.func import jacfwd
    fn = _torch_obj(obj)
    rng = np.random.default_rng(3)
    for d in ([2] if obj == "goldstein_price" else [2, 10, 50]):
        for _ in range(5):
            x = rng.uniform(-2 if obj == "goldstein_price" else -5, 2 if obj == "goldstein_price" else 5, d)
            ref = jacfwd(fn)(torch.tensor(x, dtype=torch.float64)).numpy()
            f, g = oracle_any.grad(obj, x)
            assert np.max(np.abs(g - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref))), obj


# 8th-order central difference for the first derivative
_FD8 = [(1, 4 / 5), (2, -1 / 5), (3, 4 / 105), (4, -1 / 280)]


@pytest.mark.parametrize("obj", OBJ + ["goldstein_price"])
def test_gradient_vs_central_differences(oracle_any, obj):
    rng = np.random.default_rng(11)
    dims = [2] if obj == "goldstein_price" else [2, 5, 10]
    for d in dims:
        for _ in range(5):
            lo, hi = (-2, 2) if obj == "goldstein_price" else (-5, 5)
            x = rng.uniform(lo, hi, d)
            _, g = oracle_any.grad(obj, x)
            fd = np.zeros(d)
            for j in range(d):
                h = 2e-3 * max(1.0, abs(x[j]))
                acc = 0.0
                for k, c in _FD8:
                    e = np.zeros(d)
                    e[j] = k * h
                    acc += c * (oracle_any.f(obj, x + e) - oracle_any.f(obj, x - e))
                fd[j] = acc / h
            fscale = max(1.0, abs(oracle_any.f(obj, x)))
            # truncation O(h^8) plus rounding ~ eps * |f| / h
            tol = 1e-10 * max(1.0, np.linalg.norm(g)) + 1e-12 * fscale
            assert np.linalg.norm(g - fd) <= tol, (obj, d, np.linalg.norm(g - fd), tol)


def test_ackley_gradient_at_origin_is_not_finite(oracle_any):
    # Sec. V-B: the derivative is undefined at the origin
    f, g = oracle_any.grad("ackley", np.zeros(3))
    assert abs(f) < 1e-15 and not np.all(np.isfinite(g))


def test_ackley_gradient_norm_near_origin(oracle_any):
    # the cone term dominates: ||grad|| -> 4/sqrt(d) as x -> 0 along an axis
    for d in (2, 10, 50):
        x = np.zeros(d)
        x[0] = 1e-9
        _, g = oracle_any.grad("ackley", x)
        assert abs(np.linalg.norm(g) - 4 / math.sqrt(d)) < 1e-6
