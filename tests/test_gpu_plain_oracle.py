"""GPU against the plain oracle build, at the stated tolerances.

The plain build of the oracle takes the textbook order everywhere the paper
fixes none: sums strictly left to right, inverse-Hessian row products and the
rank-2 update unfused in index order, and the C library's sin, cos and exp.
None of those choices was made to match the kernels, which sum pairwise, fuse
multiply-adds and reduce sin, cos and exp their own way.  So agreement here
is agreement of two independent roundings of the same method (Alg. 2-7), and
the bars are the stated tolerances, not bit equality:
  * swarm: the same global best, bit-identical positions for at least 99.9%
    of particles (a position can only differ after a personal-best decision
    flips at a near-tie of ulp-size), personal-best values within 1e-12;
  * trajectories (first 20 iterates of starts with identical seeds, up to
    the oracle's first near-tie decision and as far as both sides went):
    within 1e-9 relative (infinity norm) for every start up to iterate 5, and
    over all 20 iterates for at least 85% of the starts.  BFGS in Rosenbrock's
    curved valley amplifies a rounding difference several-fold per step, so
    later iterates of some d = 2 starts drift apart by more than 1e-9 (up to
    2.4e-4 by iterate 19); the worst drift per iterate is printed;
  * final results: the same status and |f_gpu - f| <= 1e-6 max(1, |f|) for
    at least 99% of the starts; success rates (f - f* < 1e-4) within 0.01.
"""
import numpy as np
import pytest

from paper_2603_28770_amd import workloads as W
from tests import plain_check as PC

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Z():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_28770_amd import zeus  # raises if libzeus.so is missing
    return zeus


@pytest.fixture(scope="module")
def ctx(Z):
    c = Z.zeus_context_create(0)
    yield c
    Z.zeus_context_destroy(c)


CASES = [
    (W.ROSENBROCK_D2, None),
    (W.RASTRIGIN_D10, 512),
    (W.ROSENBROCK_D50, 64),
    (W.ACKLEY_D50, 64),
    (W.problem(name="styblinski_d13", objective="styblinski_tang", dim=13, n=1000, lower=-5.0,
               upper=5.0, iter_pso=7, iter_bfgs=1000, seed=3, request_id=5), None),
    (W.problem(name="rastrigin_d40", objective="rastrigin", dim=40, n=80, lower=-5.12,
               upper=5.12, iter_pso=4, iter_bfgs=500, seed=11), None),
]
# Goldstein-Price is not among them: its first steps throw some starts out to
# |x| ~ 20, where the octic growth of the function leaves H and g so badly
# conditioned that the two roundings differ by 1e-5 after three iterates
# (both still end at the same minimum or both non-finite).


@pytest.mark.parametrize("p,sample", CASES, ids=[c[0]["name"] for c in CASES])
def test_gpu_against_plain_oracle(Z, ctx, p, sample):
    print(f"\n[plain] {p['name']} d={p['dim']} n={p['n']} sample={sample}", flush=True)
    g = Z.zeus_minimize(ctx, p, trace_len=PC.L, pso_state=True)
    PC.check_against_plain(g, p, sample)


TWO_PI = 6.283185307179586   # 2 pi rounded to double: the objectives' constant


def _closed_form(obj, x):
    """f at 1-D points in 80-bit arithmetic, from the definitions (Sec. V-B);
    the cosine argument is the double product 2pi x that the objective
    defines."""
    xl = x.astype(np.longdouble)
    tl = (TWO_PI * x).astype(np.longdouble)
    if obj == "rastrigin":
        return np.longdouble(10) + (xl * xl - np.longdouble(10) * np.cos(tl))
    e = np.exp(np.longdouble(1))
    return (np.longdouble(-20) * np.exp(np.longdouble(-0.2) * np.sqrt(xl * xl))
            - np.exp(np.cos(tl)) + np.longdouble(20) + e)


@pytest.mark.parametrize("obj,lo,hi", [("rastrigin", -5.12, 5.12), ("rastrigin", -1000.0, 1000.0),
                                       ("ackley", -5.0, 5.0), ("ackley", -1e6, 1e6)])
def test_device_sin_cos_exp_against_extended_precision(Z, ctx, obj, lo, hi):
    """The device's cos and exp, pinned on their own: f at the seeds (no swarm
    update, no BFGS step) of Rastrigin and Ackley at d = 1, against the closed
    form in 80-bit arithmetic, to 4 ulp of the size of the terms."""
    from oracle import oracle as O
    p = W.problem(objective=obj, dim=1, n=4096, lower=lo, upper=hi, iter_pso=0, iter_bfgs=0,
                  seed=11)
    print(f"\n[transc] {obj} in [{lo:g}, {hi:g}]", flush=True)
    g = Z.zeus_minimize(ctx, p, pso_state=True)
    x = O.pso(p)["x"][:, 0]               # the seeds, from the oracle's own stream
    assert np.array_equal(g["seeds"][:, 0], x)
    ref = _closed_form(obj, x)
    if obj == "rastrigin":
        scale = 20.0 + x * x
    else:
        scale = 20.0 + np.e + 20.0 * np.exp(-0.2 * np.abs(x)) + np.e
    err = np.abs(g["f"].astype(np.longdouble) - ref).astype(np.float64) / np.spacing(scale)
    print(f"[transc]   max error {err.max():.2f} ulp of the term size", flush=True)
    assert err.max() <= 4.0
