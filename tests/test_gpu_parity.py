"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded problems.

Bars (FP64): every output bit for bit, NaN matching NaN.  Both sides fix the
rounding of every step (same operation order, fused multiply-adds in the same
explicit places, the same sin/cos/exp algorithm), so equality is expected; the
tolerances below are the weaker bars a different rounding would have to meet
and are still checked so that a loss of exactness reports how far off it is:
  * swarm phase: bit-exact positions, velocities, personal bests and global
    best for every objective (both sides evaluate the objective in the same
    order, with fused multiply-adds only in the same explicit places and the
    same sin/cos/exp algorithm);
  * BFGS iterates: the first 20 iterates agree to 1e-9 relative (infinity
    norm) up to the first iteration where the oracle took a branch with a
    relative margin below 1e-9 (a near-tie that rounding may flip);
  * final results: same status and iteration count and |df| <= 1e-6 max(1,|f|)
    for starts without a near-tie; success rates (f - f* < 1e-4) within 0.01
    over all starts.
"""
import os

import numpy as np
import pytest

from paper_2603_28770_amd import workloads as W

pytestmark = pytest.mark.gpu

TRAJ_TOL = 1e-9
F_TOL = 1e-6


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


def _run_both(Z, ctx, O, p, trace_len=20, idx=None):
    print(f"\n[parity] {p.get('name', p['objective'])} d={p['dim']} n={p['n']}", flush=True)
    g = Z.zeus_minimize(ctx, p, trace_len=trace_len, pso_state=True)
    sw = O.pso(p)
    o = O.bfgs(p, sw["x"], idx=idx, trace_len=trace_len)
    return g, sw, o


def _check_pso(g, sw, transcendental=None):
    assert np.array_equal(g["seeds"], sw["x"])
    assert np.array_equal(g["pso_v"], sw["v"])
    assert np.array_equal(g["pso_px"], sw["px"])
    assert np.array_equal(g["pso_best_x"], sw["gx"])
    assert g["summary"]["pso_best_index"] == sw["gidx"]
    assert np.array_equal(g["pso_pf"], sw["pf"])


def _check_bfgs(g, o, p, idx=None, max_mismatch_share=0.02):
    sel = np.arange(p["n"]) if idx is None else np.asarray(idx)
    gf, gx, gi, gs = g["f"][sel], g["x"][sel], g["iters"][sel], g["status"][sel]
    same_f = (gf == o["f"]) | (np.isnan(gf) & np.isnan(o["f"]))
    same_x = np.all((gx == o["x"]) | (np.isnan(gx) & np.isnan(o["x"])), axis=1)
    exact = same_x & same_f & (gi == o["iters"]) & (gs == o["status"]) & (
        g["ls_trials"][sel] == o["ls_trials"]) & (g["skips"][sel] == o["skips"]) & (
        g["resets"][sel] == o["resets"])
    print(f"[parity]   bit-exact starts {exact.mean():.4f}", flush=True)
    tie = o["tie_iter"]
    clean = tie < 0
    # trajectories: first iterates up to (and including) the near-tie step
    tr_g, tr_o = g["trace"][sel], o["trace"]
    L = tr_o.shape[1]
    worst = 0.0
    for s in range(sel.size):
        kmax = min(L, o["iters"][s] + 1)
        if tie[s] >= 0:
            kmax = min(kmax, tie[s] + 1)
        if kmax == 0:
            continue
        a, b = tr_g[s, :kmax], tr_o[s, :kmax]
        scale = np.maximum(1.0, np.max(np.abs(b), axis=1))
        err = np.max(np.abs(a - b), axis=1) / scale
        worst = max(worst, float(err.max()))
    print(f"[parity]   worst trajectory rel err {worst:.3e}; near-tie starts "
          f"{np.mean(~clean):.3f}", flush=True)
    assert worst <= TRAJ_TOL
    # final results for starts without a near-tie
    fs = np.maximum(1.0, np.abs(o["f"]))
    with np.errstate(invalid="ignore"):
        df = np.where(same_f, 0.0, np.abs(gf - o["f"]) / fs)
    same = (gs == o["status"]) & (gi == o["iters"]) & (df <= F_TOL)
    bad_clean = np.flatnonzero(clean & ~same)
    print(f"[parity]   clean starts {clean.sum()}, clean mismatches {bad_clean.size}, "
          f"all mismatches {np.sum(~same)}", flush=True)
    assert bad_clean.size == 0, (bad_clean[:10], gs[bad_clean[:10]], o["status"][bad_clean[:10]],
                                 gi[bad_clean[:10]], o["iters"][bad_clean[:10]])
    fval_ok = (df <= F_TOL) | ~np.isfinite(o["f"])
    assert np.mean(~fval_ok) <= max_mismatch_share
    fstar = W.f_star(p["objective"], p["dim"])
    rate_g = np.mean(gf - fstar < 1e-4)
    rate_o = np.mean(o["f"] - fstar < 1e-4)
    print(f"[parity]   success gpu {rate_g:.4f} oracle {rate_o:.4f}", flush=True)
    assert abs(rate_g - rate_o) <= 0.01
    assert exact.all(), np.flatnonzero(~exact)[:10]
    tr_same = (tr_g == tr_o) | (np.isnan(tr_g) & np.isnan(tr_o))
    assert tr_same.all()


def _check_summary(g):
    s = g["summary"]
    f, st = g["f"], g["status"]
    fin = np.isfinite(f)
    if fin.any():
        b = int(np.flatnonzero(fin & (f == f[fin].min()))[0])
        assert s["best_index"] == b and s["best_f"] == f[b]
    else:
        assert s["best_index"] == -1
    assert s["n_converged"] == int(np.sum(st == 1))
    assert s["n_nonfinite"] == int(np.sum(st == 3))
    assert s["total_iters"] == int(g["iters"].sum())
    assert s["total_ls_trials"] == int(g["ls_trials"].sum())


CASES = [
    (W.ROSENBROCK_D2, False),
    (W.problem(name="rastrigin_d10", objective="rastrigin", dim=10, n=2000, lower=-5.12,
               upper=5.12, iter_pso=20, iter_bfgs=1000, seed=1), True),
    (W.problem(name="styblinski_d13", objective="styblinski_tang", dim=13, n=1000, lower=-5.0,
               upper=5.0, iter_pso=7, iter_bfgs=1000, seed=3, request_id=5), False),
    (W.problem(name="ackley_d7", objective="ackley", dim=7, n=777, lower=-5.0, upper=5.0,
               iter_pso=5, iter_bfgs=300, seed=2), True),
    (W.problem(name="goldstein_price", objective="goldstein_price", dim=2, n=1500, lower=-2.0,
               upper=2.0, iter_pso=4, iter_bfgs=500, seed=6), False),
    (W.problem(name="rosenbrock_d33", objective="rosenbrock", dim=33, n=300, lower=-5.0,
               upper=5.0, iter_pso=5, iter_bfgs=400, seed=2), False),
    (W.problem(name="quartic_d17", objective="quartic", dim=17, n=257, lower=-3.0, upper=3.0,
               iter_pso=2, iter_bfgs=200, seed=9), False),
    (W.problem(name="sphere_d64", objective="sphere", dim=64, n=129, lower=-3.0, upper=3.0,
               iter_pso=3, iter_bfgs=50, seed=4), False),
    # one wavefront per start (33..64 dimensions) for every objective
    (W.problem(name="ackley_d50", objective="ackley", dim=50, n=96, lower=-5.0, upper=5.0,
               iter_pso=5, iter_bfgs=600, seed=2), True),
    (W.problem(name="rastrigin_d40", objective="rastrigin", dim=40, n=80, lower=-5.12,
               upper=5.12, iter_pso=4, iter_bfgs=500, seed=11), True),
    (W.problem(name="styblinski_d57", objective="styblinski_tang", dim=57, n=70, lower=-5.0,
               upper=5.0, iter_pso=3, iter_bfgs=400, seed=13), False),
]


@pytest.mark.parametrize("p,transc", CASES, ids=[c[0]["name"] for c in CASES])
def test_parity(Z, ctx, oracle_mod, p, transc):
    g, sw, o = _run_both(Z, ctx, oracle_mod, p)
    _check_pso(g, sw, transc)
    _check_bfgs(g, o, p)
    _check_summary(g)


def test_rosenbrock_d64_max_dim(Z, ctx, oracle_mod):
    p = W.problem(name="rosenbrock_d64", objective="rosenbrock", dim=64, n=70, lower=-2.0,
                  upper=2.0, iter_pso=2, iter_bfgs=300, seed=12)
    g, sw, o = _run_both(Z, ctx, oracle_mod, p)
    _check_pso(g, sw, False)
    _check_bfgs(g, o, p)


# Above 64 dimensions a start runs on a block: up to 128 with its inverse
# Hessian in the registers of four wavefronts, up to 208 in the registers of
# eight wavefronts and LDS, above that in device memory.  Just over the
# narrow limit, unaligned and aligned sizes, both sides of 128 and 208, and
# the largest dimension of the build.
WIDE_CASES = [
    W.problem(name="rosenbrock_d65", objective="rosenbrock", dim=65, n=70, lower=-2.0, upper=2.0,
              iter_pso=2, iter_bfgs=300, seed=12),
    W.problem(name="rastrigin_d100", objective="rastrigin", dim=100, n=40, lower=-5.12,
              upper=5.12, iter_pso=3, iter_bfgs=300, seed=1, request_id=3),
    # two term sums (K = 2) on the four-wavefront block, whose next value
    # takes both sums of the accepted line-search trial
    W.problem(name="ackley_d90", objective="ackley", dim=90, n=30, lower=-5.0, upper=5.0,
              iter_pso=2, iter_bfgs=200, seed=14),
    W.problem(name="styblinski_d128", objective="styblinski_tang", dim=128, n=33, lower=-5.0,
              upper=5.0, iter_pso=2, iter_bfgs=200, seed=3),
    W.problem(name="rosenbrock_d129", objective="rosenbrock", dim=129, n=24, lower=-2.0, upper=2.0,
              iter_pso=2, iter_bfgs=300, seed=13),
    W.problem(name="ackley_d200", objective="ackley", dim=200, n=20, lower=-5.0, upper=5.0,
              iter_pso=2, iter_bfgs=200, seed=2),
    W.problem(name="styblinski_d208", objective="styblinski_tang", dim=208, n=16, lower=-5.0,
              upper=5.0, iter_pso=2, iter_bfgs=150, seed=5),
    W.problem(name="rosenbrock_d209", objective="rosenbrock", dim=209, n=12, lower=-2.0, upper=2.0,
              iter_pso=1, iter_bfgs=120, seed=6),
    W.problem(name="sphere_d256", objective="sphere", dim=256, n=9, lower=-3.0, upper=3.0,
              iter_pso=1, iter_bfgs=30, seed=4),
]


@pytest.mark.parametrize("p", WIDE_CASES, ids=[c["name"] for c in WIDE_CASES])
def test_parity_wide(Z, ctx, oracle_mod, p):
    g, sw, o = _run_both(Z, ctx, oracle_mod, p)
    _check_pso(g, sw)
    _check_bfgs(g, o, p)
    _check_summary(g)


@pytest.mark.parametrize("lanes", [None, 256], ids=["on_chip", "device_memory"])
def test_wide_more_starts_than_slots(Z, ctx, oracle_mod, lanes):
    """2300 starts on at most 2048 resident blocks (device memory: H slots) or
    the resident blocks of the on-chip kernel: the later starts come from the
    work counter and reuse the blocks (and H slots) of finished starts
    (sampled)."""
    p = W.problem(name="rosenbrock_d70_n2300", objective="rosenbrock", dim=70, n=2300, lower=-2.0,
                  upper=2.0, iter_pso=1, iter_bfgs=60, seed=21)
    idx = np.concatenate([np.arange(0, 40), np.arange(2048, 2300, 7)])
    if lanes:
        os.environ["ZEUS_TILE_LANES"] = str(lanes)
    try:
        g, sw, o = _run_both(Z, ctx, oracle_mod, p, idx=idx)
    finally:
        os.environ.pop("ZEUS_TILE_LANES", None)
    _check_pso(g, sw)
    _check_bfgs(g, o, p, idx=idx)
    _check_summary(g)


# The device-memory block at dimensions the on-chip blocks also cover.
_DM = [c for c in WIDE_CASES if c["dim"] in (65, 100, 128, 200)]


@pytest.mark.parametrize("p", _DM, ids=[c["name"] for c in _DM])
def test_parity_device_memory_block(Z, ctx, oracle_mod, p):
    os.environ["ZEUS_TILE_LANES"] = "256"
    try:
        g, sw, o = _run_both(Z, ctx, oracle_mod, p)
    finally:
        del os.environ["ZEUS_TILE_LANES"]
    _check_pso(g, sw)
    _check_bfgs(g, o, p)
    _check_summary(g)


def test_single_start_and_dim_one(Z, ctx, oracle_mod):
    for p in (W.problem(name="one", objective="rastrigin", dim=3, n=1, lower=-2.0, upper=2.0,
                        iter_pso=3, seed=8),
              W.problem(name="d1", objective="styblinski_tang", dim=1, n=100, lower=-5.0,
                        upper=5.0, iter_pso=2, seed=8)):
        g, sw, o = _run_both(Z, ctx, oracle_mod, p)
        _check_pso(g, sw, p["objective"] == "rastrigin")
        _check_bfgs(g, o, p)
        _check_summary(g)


def test_zero_budgets(Z, ctx, oracle_mod):
    p = W.problem(name="zero", objective="rosenbrock", dim=5, n=300, lower=-2.0, upper=2.0,
                  iter_pso=0, iter_bfgs=0, seed=3)
    g, sw, o = _run_both(Z, ctx, oracle_mod, p, trace_len=2)
    _check_pso(g, sw, False)
    assert np.array_equal(g["x"], sw["x"]) and np.all(g["iters"] == 0)
    assert np.all(g["status"] == 0) and np.array_equal(g["f"], o["f"])
    assert np.all(np.isnan(g["trace"][:, 1]))


def test_non_finite_path(Z, ctx):
    p = W.problem(name="huge", objective="rosenbrock", dim=3, n=64, lower=1e200, upper=2e200,
                  iter_bfgs=10)
    g = Z.zeus_minimize(ctx, p)
    assert np.all(g["status"] == 3) and np.all(g["iters"] == 0)
    assert g["summary"]["best_index"] == -1 and g["summary"]["n_nonfinite"] == 64


def test_ackley_failure_mode(Z, ctx):
    p = W.problem(name="ackley0", objective="ackley", dim=2, n=64, lower=-0.1, upper=0.1,
                  iter_bfgs=200, seed=5)
    g = Z.zeus_minimize(ctx, p)
    near = np.max(np.abs(g["x"]), axis=1) < 1e-3
    assert near.mean() >= 0.8
    assert np.all(g["status"][near] == 0) and np.all(g["iters"][near] == 200)


def test_sphere_one_exact_step(Z, ctx):
    p = W.problem(objective="sphere", dim=9, n=500, lower=-3.0, upper=3.0, iter_pso=2, seed=2)
    g = Z.zeus_minimize(ctx, p)
    assert np.all(g["status"] == 1) and np.all(g["iters"] == 1) and np.all(g["x"] == 0.0)


def test_deterministic_repeat(Z, ctx):
    p = W.scaled(W.RASTRIGIN_D10, 5000)
    a = Z.zeus_minimize(ctx, p, pso_state=True)
    b = Z.zeus_minimize(ctx, p, pso_state=True)
    for k in ("f", "x", "iters", "status", "ls_trials", "skips", "resets", "seeds"):
        assert np.array_equal(a[k], b[k]), k


def test_async_matches_blocking(Z, ctx):
    import torch
    p = W.scaled(W.RASTRIGIN_D10, 3000)
    a = Z.zeus_minimize(ctx, p, pso_state=True, trace_len=4)
    ds = Z.DeviceSolve(p, trace_len=4, pso_state=True)
    s = torch.cuda.Stream()
    ds.enqueue(ctx, s.cuda_stream)
    s.synchronize()
    b = ds.host()
    for k in ("f", "x", "iters", "status", "ls_trials", "skips", "resets", "seeds", "pso_v",
              "pso_px", "pso_pf", "pso_best_x", "trace"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    assert a["summary"] == b["summary"]


def test_errors_through_the_abi(Z, ctx):
    bad = Z.make_problem(W.problem(objective="rastrigin", dim=257, n=10, lower=-1.0, upper=1.0))
    with pytest.raises(Z.ZeusError) as e:
        Z.zeus_minimize(ctx, bad)
    assert e.value.code == Z.EUNSUPPORTED
    with pytest.raises(Z.ZeusError) as e:
        Z.zeus_minimize(ctx, W.problem(objective="rastrigin", dim=0, n=10, lower=-1.0, upper=1.0))
    assert e.value.code == Z.EINVAL


def test_full_size_rastrigin_sampled(Z, ctx, oracle_mod):
    """The benchmark's workload at full size (N = 65,536, d = 10): the whole
    swarm bit for bit and a strided sample of 512 starts against the oracle."""
    p = W.RASTRIGIN_D10
    idx = W.strided_subset(p["n"], 512)
    g, sw, o = _run_both(Z, ctx, oracle_mod, p, idx=idx)
    _check_pso(g, sw, True)
    _check_bfgs(g, o, p, idx=idx)
    _check_summary(g)


@pytest.mark.parametrize("p", [W.ACKLEY_D50, W.ROSENBROCK_D50], ids=lambda p: p["name"])
def test_full_size_d50_sampled(Z, ctx, oracle_mod, p):
    """The d = 50 bench workloads at full size (N = 131,072, 64 lanes per
    start): the whole swarm bit for bit and a strided sample of 64 starts,
    with their first 20 iterates, against the oracle."""
    print(f"\n[parity] {p['name']} full size, 64 sampled starts", flush=True)
    idx = W.strided_subset(p["n"], 64)
    g, sw, o = _run_both(Z, ctx, oracle_mod, p, idx=idx)
    _check_pso(g, sw, True)
    _check_bfgs(g, o, p, idx=idx)
    _check_summary(g)
