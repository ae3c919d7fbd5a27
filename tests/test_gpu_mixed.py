"""Mixed precision on the GPU (objective and dual numbers in FP32; inverse
Hessian, search direction, g'p, the Armijo comparison, s, y and y's in FP64)
against the FP64 oracle on the same problems.  The bars are the ones stated
for this mode: the swarm is FP64 in both and must match bit for bit; success
rates (f - f* < 1e-4, f re-evaluated in FP64 at the returned x) agree within
0.01; and the error of each start against the oracle is reported, with most
starts ending at the oracle's minimum to within FP32 noise."""
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
    (dict(W.ROSENBROCK_D2, grad_tol=1e-4), 0.95),
    (W.problem(name="st_d5", objective="styblinski_tang", dim=5, n=3000, lower=-5.0, upper=5.0,
               iter_pso=3, iter_bfgs=500, grad_tol=1e-4, seed=7), 0.8),
    (W.problem(name="rastrigin_d3", objective="rastrigin", dim=3, n=3000, lower=-5.12,
               upper=5.12, iter_pso=10, iter_bfgs=500, grad_tol=1e-4, seed=4), 0.8),
    (W.problem(name="ackley_d5", objective="ackley", dim=5, n=2000, lower=-5.0, upper=5.0,
               iter_pso=5, iter_bfgs=300, grad_tol=1e-4, seed=3), 0.6),
    (dict(W.scaled(W.RASTRIGIN_D10, 4000), grad_tol=1e-4), 0.6),
    (W.problem(name="rosenbrock_d20", objective="rosenbrock", dim=20, n=500, lower=-2.0,
               upper=2.0, iter_pso=3, iter_bfgs=2000, grad_tol=1e-4, seed=8), 0.8),
    # above 64 dimensions (one block of 256 lanes per start)
    (W.problem(name="styblinski_d96", objective="styblinski_tang", dim=96, n=200, lower=-5.0,
               upper=5.0, iter_pso=2, iter_bfgs=500, grad_tol=1e-4, seed=5), 0.6),
    (W.problem(name="rosenbrock_d72", objective="rosenbrock", dim=72, n=300, lower=-2.0,
               upper=2.0, iter_pso=2, iter_bfgs=4000, grad_tol=1e-4, seed=9), 0.7),
]


@pytest.mark.parametrize("p,min_same", CASES, ids=[c[0].get("name", "p") for c in CASES])
def test_mixed_against_fp64_oracle(Z, ctx, oracle_mod, p, min_same):
    pm = dict(p, precision="mixed")
    print(f"\n[mixed] {p.get('name')} d={p['dim']} n={p['n']}", flush=True)
    g = Z.zeus_minimize(ctx, pm, pso_state=True)
    sw = oracle_mod.pso(p)
    o = oracle_mod.bfgs(p, sw["x"])
    assert np.array_equal(g["seeds"], sw["x"]) and np.array_equal(g["pso_pf"], sw["pf"])
    # reported f is the FP64 value at the returned x
    for i in range(0, p["n"], max(1, p["n"] // 25)):
        if np.isfinite(g["f"][i]):
            assert g["f"][i] == oracle_mod.f(p["objective"], g["x"][i])
    fs = np.maximum(1.0, np.abs(o["f"]))
    df = np.abs(g["f"] - o["f"]) / fs
    dx = np.max(np.abs(g["x"] - o["x"]), axis=1) / np.maximum(1.0, np.max(np.abs(o["x"]), axis=1))
    same = df <= 1e-4
    fstar = W.f_star(p["objective"], p["dim"])
    rg, ro = np.mean(g["f"] - fstar < 1e-4), np.mean(o["f"] - fstar < 1e-4)
    print(f"[mixed]   same minimum {same.mean():.3f}; |df| p50 {np.median(df):.2e} "
          f"p90 {np.quantile(df, 0.9):.2e}; |dx| p50 {np.median(dx):.2e}; "
          f"converged gpu {np.mean(g['status'] == 1):.3f} oracle {np.mean(o['status'] == 1):.3f}; "
          f"success gpu {rg:.4f} oracle {ro:.4f}", flush=True)
    assert same.mean() >= min_same
    assert abs(rg - ro) <= 0.01


@pytest.mark.parametrize("p", [W.ROSENBROCK_D50, W.ACKLEY_D50], ids=lambda p: p["name"])
def test_mixed_d50_full_size(Z, ctx, oracle_mod, p):
    """The d = 50 workloads in mixed precision at full size (N = 131,072, the
    64-lane FP32 kernel with FP64 H), against the FP64 oracle on a strided
    sample of 512 starts and against the FP64 GPU solve on every start.
    The swarm is FP64 on both sides and matches bit for bit; the reported f
    is the FP64 value at the returned x; on the sample most starts end at the
    oracle's minimum and the success rates (f - f* < 1e-4) agree within 0.02
    (ten starts of 512); over all starts the mixed solve's success rate is
    within 0.01 of the FP64 solve's."""
    pm = dict(p, precision="mixed", grad_tol=1e-4)
    print(f"\n[mixed] {p['name']} full size, 512 sampled starts", flush=True)
    g = Z.zeus_minimize(ctx, pm, pso_state=True)
    g64 = Z.zeus_minimize(ctx, p)
    idx = W.strided_subset(p["n"], 512)
    sw = oracle_mod.pso(p)
    assert np.array_equal(g["seeds"], sw["x"]) and np.array_equal(g["pso_pf"], sw["pf"])
    o = oracle_mod.bfgs(p, sw["x"], idx=idx)
    gf, gx = g["f"][idx], g["x"][idx]
    for k in range(0, idx.size, 16):
        if np.isfinite(gf[k]):
            assert gf[k] == oracle_mod.f(p["objective"], gx[k])
    df = np.abs(gf - o["f"]) / np.maximum(1.0, np.abs(o["f"]))
    same = df <= 1e-4
    fstar = W.f_star(p["objective"], p["dim"])
    rs, ro = np.mean(gf - fstar < 1e-4), np.mean(o["f"] - fstar < 1e-4)
    rg, r64 = np.mean(g["f"] - fstar < 1e-4), np.mean(g64["f"] - fstar < 1e-4)
    print(f"[mixed]   sample: same minimum {same.mean():.3f}, |df| p50 {np.median(df):.2e} "
          f"p90 {np.quantile(df, 0.9):.2e}, success gpu {rs:.4f} oracle {ro:.4f}; "
          f"all starts: success mixed {rg:.4f} fp64 {r64:.4f}; iterations mixed "
          f"{int(np.sum(g['iters']))} fp64 {int(np.sum(g64['iters']))}", flush=True)
    assert same.mean() >= 0.8
    assert abs(rs - ro) <= 0.02
    assert abs(rg - r64) <= 0.01
