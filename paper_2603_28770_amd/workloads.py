"""Seeded synthetic workloads (problem parameter sets).

This module only describes inputs: objective, box, sizes, budgets, seeds.  It
holds none of the method's arithmetic; the random numbers the method itself
draws come from the counter-based Philox stream keyed by (seed, request_id),
which the GPU library and the oracle each implement on their own.

Problems are plain dicts with the field names of ``zeus_problem``; missing
fields take the paper's defaults (PSO w=0.5, c1=1.2, c2=1.5 from Sec. III-A;
Armijo c=0.3 and 20 trials from Sec. III-D; velocity half-range upper-lower
from Alg. 2).
"""
import math

import numpy as np

PAPER_DEFAULTS = dict(iter_pso=0, w=0.5, c1=1.2, c2=1.5, v_half=0.0, iter_bfgs=1000,
                      iter_ls=20, armijo_c=0.3, ls_shrink=0.5, grad_tol=1e-6, seed=0,
                      request_id=0, precision="fp64")

# Objective minima used for the success criterion f - f* < 1e-4.
# Styblinski-Tang: x* is the root of 4x^3 - 32x + 5 = 0 near -2.9035.
ST_XSTAR = -2.903534027771178
ST_FSTAR_PER_DIM = -39.16616570377141


def f_star(objective: str, dim: int) -> float:
    return {"rosenbrock": 0.0, "rastrigin": 0.0, "ackley": 0.0, "sphere": 0.0, "quartic": 0.0,
            "goldstein_price": 3.0, "styblinski_tang": ST_FSTAR_PER_DIM * dim}[objective]


def x_star(objective: str, dim: int) -> np.ndarray:
    if objective == "rosenbrock":
        return np.ones(dim)
    if objective == "goldstein_price":
        return np.array([0.0, -1.0])
    if objective == "styblinski_tang":
        return np.full(dim, ST_XSTAR)
    return np.zeros(dim)


def problem(**kw) -> dict:
    p = dict(PAPER_DEFAULTS)
    p.update(kw)
    return p


# Rosenbrock, d=2, N=1024 in [-5,5]^2, seed 0; PSO 10 iterations with
# w=0.7, c1=c2=1.5, v0 in [-1,1]; BFGS <= 100, Armijo c=1e-4, Theta=1e-6.
ROSENBROCK_D2 = problem(name="rosenbrock_d2_n1024", objective="rosenbrock", dim=2, n=1024,
                        lower=-5.0, upper=5.0, iter_pso=10, w=0.7, c1=1.5, c2=1.5, v_half=1.0,
                        iter_bfgs=100, armijo_c=1e-4, grad_tol=1e-6, seed=0)

# Rastrigin, d=10, N=65,536 in [-5.12,5.12]^10, seed 1; PSO 20 (paper's
# coefficients), BFGS <= 1000; Theta 1e-6 (fp64) or 1e-4 (mixed).
RASTRIGIN_D10 = problem(name="rastrigin_d10_n65536", objective="rastrigin", dim=10, n=65536,
                        lower=-5.12, upper=5.12, iter_pso=20, iter_bfgs=1000, grad_tol=1e-6,
                        seed=1)
RASTRIGIN_D10_MIXED = dict(RASTRIGIN_D10, name="rastrigin_d10_n65536_mixed", grad_tol=1e-4,
                           precision="mixed")

# Ackley and Rosenbrock, d=50, N=131,072 in [-5,5]^50, seed 2; PSO 5, BFGS <= 2000.
ACKLEY_D50 = problem(name="ackley_d50_n131072", objective="ackley", dim=50, n=131072,
                     lower=-5.0, upper=5.0, iter_pso=5, iter_bfgs=2000, seed=2)
ROSENBROCK_D50 = problem(name="rosenbrock_d50_n131072", objective="rosenbrock", dim=50,
                         n=131072, lower=-5.0, upper=5.0, iter_pso=5, iter_bfgs=2000, seed=2)

# Wide problems (one block per start): Styblinski-Tang and Rosenbrock,
# d = 128, N = 16,384 in [-5,5]^128, seed 5; PSO 2, BFGS <= 1000.
STYBLINSKI_D128 = problem(name="styblinski_d128_n16384", objective="styblinski_tang", dim=128,
                          n=16384, lower=-5.0, upper=5.0, iter_pso=2, iter_bfgs=1000, seed=5)
ROSENBROCK_D128 = problem(name="rosenbrock_d128_n16384", objective="rosenbrock", dim=128,
                          n=16384, lower=-5.0, upper=5.0, iter_pso=2, iter_bfgs=1000, seed=5)

ROSENBROCK_D200 = problem(name="rosenbrock_d200_n8192", objective="rosenbrock", dim=200, n=8192,
                          lower=-5.0, upper=5.0, iter_pso=2, iter_bfgs=2000, seed=5)

# User-code objectives (compiled at run time): Rosenbrock restated as user
# code on the d = 50 problem above (same box, seed and budgets; also in mixed
# precision with Theta 1e-4), on the
# d = 200 problem with L-BFGS keeping 8 pairs, and the
# synthetic binned Poisson-likelihood fit, 4 parameters in [0,10]^4,
# N = 65,536, seed 6; PSO 10, BFGS <= 1000.
USER_ROSENBROCK_D50 = dict(ROSENBROCK_D50, name="user_rosenbrock_d50_n131072", objective="user")
USER_ROSENBROCK_D50_MIXED = dict(USER_ROSENBROCK_D50, name="user_rosenbrock_d50_n131072_mixed",
                                 precision="mixed", grad_tol=1e-4)
USER_ROSENBROCK_D200_LBFGS = dict(ROSENBROCK_D200, name="user_rosenbrock_d200_n8192_lbfgs8",
                                  objective="user", lbfgs_m=8)
USER_POISSON_FIT = problem(name="user_poisson_fit_n65536", objective="user", dim=4, n=65536,
                           lower=0.0, upper=10.0, iter_pso=10, iter_bfgs=1000, seed=6)

BOXES = {"rosenbrock": (-5.0, 5.0), "ackley": (-5.0, 5.0), "styblinski_tang": (-5.0, 5.0),
         "rastrigin": (-5.12, 5.12)}
MIX = ("rosenbrock", "rastrigin", "ackley", "styblinski_tang")


def _request_stream(seed: int, count: int, dmax_span: int, nmin: int):
    """Uniforms for the request generator: numpy Philox keyed (seed, 'REQ')."""
    tag = int.from_bytes(b"REQ", "little")
    g = np.random.Generator(np.random.Philox(key=[seed, tag]))
    u = g.random((count, 4))
    out = []
    for r in range(count):
        obj = MIX[min(int(u[r, 0] * 4), 3)]
        d = 2 + int(u[r, 1] * dmax_span)
        n = int(nmin * 64.0 ** u[r, 2])
        ipso = int(u[r, 3] * 21)
        lo, hi = BOXES[obj]
        dim = max(d, 2)
        out.append(problem(name=f"req{r}", objective=obj, dim=dim, n=n, lower=lo, upper=hi,
                           iter_pso=ipso, iter_bfgs=1000, seed=seed, request_id=r))
    return out


def uneven_batch(count: int = 512, seed: int = 3):
    """512 requests: objective uniform over the mix, d uniform in [2,128],
    N log-uniform in [256, 16384], PSO iterations uniform in [0,20], BFGS <= 1000."""
    return _request_stream(seed, count, 127, 256)


def served_mix(count: int = 4096, seed: int = 4):
    """4,096 requests: as the uneven batch with d in [2,200], N log-uniform in
    [1024, 65536]; mixed precision, Theta 1e-4."""
    reqs = _request_stream(seed, count, 199, 1024)
    for r in reqs:
        r.update(precision="mixed", grad_tol=1e-4)
    return reqs


def footprint_bytes(p: dict) -> int:
    """Resident state per request, N (8 d^2 + 32 d) bytes: one d x d fp64
    inverse Hessian and four fp64 d-vectors per start."""
    d, n = int(p["dim"]), int(p["n"])
    return n * (8 * d * d + 32 * d)


def scaled(p: dict, n: int, **kw) -> dict:
    """The same problem with fewer starts (and optional overrides)."""
    q = dict(p)
    q["n"] = int(n)
    q.update(kw)
    q["name"] = f"{p.get('name', 'problem')}_n{n}"
    return q


def strided_subset(n: int, count: int) -> np.ndarray:
    """Deterministic strided subset of start indices: every ceil(n/count)-th."""
    step = max(1, math.ceil(n / count))
    return np.arange(0, n, step, dtype=np.int64)
