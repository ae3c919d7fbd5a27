"""The effectiveness-study figures (N_correct, the end-point groups) from a
GPU run equal those of the oracle on the same run: a small version of each
study configuration (Rastrigin by dimension with 5 sweeps; d = 5 Rastrigin
and Rosenbrock by number of sweeps), each stopped at 100 convergences."""
import numpy as np
import pytest

from paper_2603_28770_amd import studies as S

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


CASES = [("rastrigin", 2, 5, 11), ("rastrigin", 7, 5, 12), ("rastrigin", 5, 0, 13),
         ("rastrigin", 5, 20, 14), ("rosenbrock", 5, 2, 15)]


@pytest.mark.parametrize("obj,d,sweeps,seed", CASES)
def test_study_run_matches_oracle(Z, ctx, oracle_mod, obj, d, sweeps, seed):
    print(f"\n[study] {obj} d={d} sweeps={sweeps} seed={seed}", flush=True)
    p = S.study_problem(obj, d, 3000, sweeps, seed, 100)
    g = Z.zeus_minimize(ctx, p, ls_trials=False)
    x0 = oracle_mod.pso(p)["x"]
    o, _ = oracle_mod.bfgs_required(p, x0, 100)
    for k in ("f", "x", "status"):
        assert np.array_equal(g[k], o[k], equal_nan=True), k
    o["summary"] = {"best_f": float(np.min(np.where(np.isfinite(o["f"]), o["f"], np.inf)))}
    assert S.run_summary(g, obj) == S.run_summary(o, obj)
