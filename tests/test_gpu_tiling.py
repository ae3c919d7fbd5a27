"""Every tiling of the BFGS phase (2..64 lanes per start, or one block per
start with H in its registers up to d = 128, in its registers and LDS up to
d = 208, or in device memory) returns bit-identical results: they evaluate the
same pairwise sums.  Forced through ZEUS_TILE_LANES."""
import os

import numpy as np
import pytest

from paper_2603_28770_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Z():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_28770_amd import zeus
    return zeus


@pytest.fixture(scope="module")
def ctx(Z):
    c = Z.zeus_context_create(0)
    yield c
    Z.zeus_context_destroy(c)


CASES = [
    W.problem(name="rast3", objective="rastrigin", dim=3, n=500, lower=-5.12, upper=5.12,
              iter_pso=3, iter_bfgs=200, seed=3),
    W.problem(name="ros11", objective="rosenbrock", dim=11, n=300, lower=-2.0, upper=2.0,
              iter_pso=2, iter_bfgs=400, seed=4),
    W.problem(name="ack40_mixed", objective="ackley", dim=40, n=200, lower=-5.0, upper=5.0,
              iter_pso=2, iter_bfgs=300, seed=5, precision="mixed", grad_tol=1e-4),
    W.problem(name="ros90", objective="rosenbrock", dim=90, n=60, lower=-2.0, upper=2.0,
              iter_pso=2, iter_bfgs=250, seed=6),
    W.problem(name="rast120_mixed", objective="rastrigin", dim=120, n=40, lower=-5.12, upper=5.12,
              iter_pso=2, iter_bfgs=200, seed=7, precision="mixed", grad_tol=1e-4),
    W.problem(name="ros150", objective="rosenbrock", dim=150, n=24, lower=-2.0, upper=2.0,
              iter_pso=2, iter_bfgs=200, seed=8),
    W.problem(name="ack170_mixed", objective="ackley", dim=170, n=16, lower=-5.0, upper=5.0,
              iter_pso=2, iter_bfgs=150, seed=9, precision="mixed", grad_tol=1e-4),
]


@pytest.mark.parametrize("p", CASES, ids=[c["name"] for c in CASES])
def test_all_tilings_agree(Z, ctx, p):
    g = 4
    while g < p["dim"]:
        g *= 2
    tilings = []
    while g <= 64:
        tilings.append(g)
        g *= 2
    if p["dim"] <= 128:
        tilings.append(128)  # one block per start, H in its wavefronts' registers
    if p["dim"] <= 208:
        tilings.append(208)  # one block per start, H in its registers and LDS
    tilings.append(256)      # one block per start, H in device memory
    ref = None
    for lanes in tilings:
        print(f"\n[tiling] {p['name']} lanes={lanes}", flush=True)
        os.environ["ZEUS_TILE_LANES"] = str(lanes)
        try:
            out = Z.zeus_minimize(ctx, p)
        finally:
            del os.environ["ZEUS_TILE_LANES"]
        if ref is None:
            ref = out
            continue
        for k in ("f", "x", "iters", "status", "ls_trials", "skips", "resets"):
            assert np.array_equal(ref[k], out[k], equal_nan=True), (lanes, k)
