"""Results do not depend on how many workers share the starts, nor on which
worker runs which start, and a solve repeated gives the same bits.  The
persistent BFGS kernels size their grid from the compute units;
ZEUS_BFGS_CUS sizes it for fewer, so the same starts run on a handful of
lane groups or blocks (claimed in a different order from the work counter)
instead of the whole chip.  Covers every BFGS kernel, L-BFGS and the two
early-stop passes (whose second pass splits the starts statically by
worker)."""
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
    W.problem(name="rast10_lanes16", objective="rastrigin", dim=10, n=3000, lower=-5.12,
              upper=5.12, iter_pso=3, iter_bfgs=300, seed=31),
    W.problem(name="ros50_lanes64", objective="rosenbrock", dim=50, n=300, lower=-2.0, upper=2.0,
              iter_pso=2, iter_bfgs=600, seed=32),
    W.problem(name="ros100_four_waves", objective="rosenbrock", dim=100, n=40, lower=-2.0,
              upper=2.0, iter_pso=2, iter_bfgs=300, seed=33),
    W.problem(name="ack150_eight_waves", objective="ackley", dim=150, n=20, lower=-5.0, upper=5.0,
              iter_pso=2, iter_bfgs=150, seed=34),
    W.problem(name="st120_lbfgs", objective="styblinski_tang", dim=120, n=80, lower=-5.0,
              upper=5.0, iter_pso=2, iter_bfgs=300, seed=35, lbfgs_m=4),
    W.problem(name="rast5_early_stop", objective="rastrigin", dim=5, n=4000, lower=-5.12,
              upper=5.12, iter_pso=2, iter_bfgs=200, seed=36, required_converged=40),
]
KEYS = ("f", "x", "iters", "status", "ls_trials", "skips", "resets")


def _timed(Z, ctx, p):
    """The solve and its BFGS kernels' time (HIP events)."""
    Z.zeus_context_set_profiling(ctx, True)
    try:
        out = Z.zeus_minimize(ctx, p)
        ms = Z.zeus_context_get_profile(ctx)["bfgs_ms"]
    finally:
        Z.zeus_context_set_profiling(ctx, False)
    return out, ms


@pytest.mark.parametrize("p", CASES, ids=[c["name"] for c in CASES])
def test_worker_count_and_repeat_invariance(Z, ctx, p):
    print(f"\n[workers] {p['name']} default grid", flush=True)
    ref = Z.zeus_minimize(ctx, p)  # also loads the kernels before anything is timed
    again, ms_full = _timed(Z, ctx, p)
    for k in KEYS:
        assert np.array_equal(ref[k], again[k], equal_nan=True), ("repeat", k)
    for cus in (1, 3):
        print(f"[workers] {p['name']} grid of {cus} compute units", flush=True)
        os.environ["ZEUS_BFGS_CUS"] = str(cus)
        try:
            out, ms = _timed(Z, ctx, p)
        finally:
            del os.environ["ZEUS_BFGS_CUS"]
        for k in KEYS:
            assert np.array_equal(ref[k], out[k], equal_nan=True), (cus, k)
        assert ref["summary"]["best_f"] == out["summary"]["best_f"]
        if cus == 1:  # the grid did shrink: the same starts on far fewer workers
            assert ms > 1.5 * ms_full, (ms, ms_full)
