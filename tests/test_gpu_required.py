"""Early stop (required_converged = c > 0, Alg. 10) on the GPU against the
oracle's reading of it (every start still running when the c-th start
converges stops there), bit for bit: through every entry point (blocking,
batch, server, asynchronous, allocation-free, graph-captured), with several
early-stop requests in one launch group, with L-BFGS and at full size."""
import numpy as np
import pytest

from paper_2603_28770_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("f", "x", "iters", "status", "ls_trials", "skips", "resets")


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
    (W.problem(name="rast4", objective="rastrigin", dim=4, n=300, lower=-5.12, upper=5.12,
               iter_pso=3, iter_bfgs=200, seed=8), 37),
    (W.problem(name="ros5", objective="rosenbrock", dim=5, n=500, lower=-2.0, upper=2.0,
               iter_pso=2, iter_bfgs=500, seed=3), 1),
    (W.problem(name="ros2_c100", objective="rosenbrock", dim=2, n=1024, lower=-5.0, upper=5.0,
               iter_pso=10, w=0.7, c1=1.5, c2=1.5, v_half=1.0, iter_bfgs=100, armijo_c=1e-4,
               seed=0), 100),
    (W.problem(name="st3_never", objective="styblinski_tang", dim=3, n=200, lower=-5.0, upper=5.0,
               iter_pso=1, iter_bfgs=5, seed=2), 150),
    (W.problem(name="ack70_wide", objective="ackley", dim=70, n=40, lower=-2.0, upper=2.0,
               iter_pso=1, iter_bfgs=300, seed=6), 10),
]


@pytest.mark.parametrize("p,c", CASES, ids=[x[0]["name"] for x in CASES])
def test_required_c_matches_oracle(Z, ctx, oracle_mod, p, c):
    print(f"\n[required] {p['name']} c={c}", flush=True)
    g = Z.zeus_minimize(ctx, dict(p, required_converged=c))
    x0 = oracle_mod.pso(p)["x"]
    o, kstar = oracle_mod.bfgs_required(p, x0, c)
    print(f"[required]   K* = {kstar}, stopped {np.sum(o['status'] == 2)}", flush=True)
    for k in KEYS:
        assert np.array_equal(g[k], o[k], equal_nan=True), k
    assert g["summary"]["n_converged"] == int(np.sum(o["status"] == 1))


def test_required_c_in_batch_and_server(Z, ctx):
    reqs = [dict(CASES[0][0], required_converged=CASES[0][1]),
            W.scaled(W.RASTRIGIN_D10, 2000),
            dict(CASES[1][0], required_converged=CASES[1][1], request_id=4)]
    alone = [Z.zeus_minimize(ctx, p) for p in reqs]
    batch = Z.zeus_minimize_batch(ctx, reqs)
    with Z.Server(ctx, 2 << 30) as srv:
        served = [srv.wait(t, timeout_s=120) for t in [srv.submit(p) for p in reqs]]
    for a, b, s in zip(alone, batch, served):
        for k in KEYS:
            assert np.array_equal(a[k], b[k], equal_nan=True) and np.array_equal(a[k], s[k], equal_nan=True)


def test_required_c_on_device_paths(Z, ctx):
    """The stop is decided on the device, so the asynchronous entry point,
    its allocation-free form and a graph-captured plan (replayed twice) give
    the blocking entry point's results bit for bit."""
    import torch
    p = dict(CASES[0][0], required_converged=CASES[0][1])
    print(f"\n[required] async / static / plan paths, {p['name']}", flush=True)
    ref = Z.zeus_minimize(ctx, p)
    ds = Z.DeviceSolve(p)
    ds.enqueue(ctx)
    torch.cuda.synchronize()
    a = ds.host()
    ds2 = Z.DeviceSolve(p)
    ds2.enqueue_static(ctx)
    torch.cuda.synchronize()
    st = ds2.host()
    plan = Z.DevicePlan(ctx, [p, dict(CASES[1][0], required_converged=CASES[1][1])])
    reps = []
    for _ in range(2):
        plan.launch()
        torch.cuda.synchronize()
        reps.append(plan.host()[0])
        Z.zeus_minimize(ctx, CASES[2][0])  # other work between the replays
    plan.close()
    for out in [a, st] + reps:
        for k in KEYS:
            assert np.array_equal(ref[k], out[k], equal_nan=True), k
        assert out["summary"]["n_converged"] == ref["summary"]["n_converged"]


def test_required_c_shared_group_and_lbfgs(Z, ctx, oracle_mod):
    """Two early-stop requests of one launch group (each with its own K*)
    beside a request without early stop, and early stop with L-BFGS, against
    the oracle."""
    reqs = [dict(CASES[0][0], required_converged=11),
            dict(CASES[0][0], required_converged=90, request_id=7, seed=9),
            dict(CASES[0][0], request_id=3),
            dict(CASES[1][0], lbfgs_m=5, required_converged=30, request_id=2)]
    print("\n[required] shared group + L-BFGS", flush=True)
    got = Z.zeus_minimize_batch(ctx, reqs)
    for p, g in zip(reqs, got):
        x0 = oracle_mod.pso(p)["x"]
        c = p.get("required_converged", 0)
        o = oracle_mod.bfgs_required(p, x0, c)[0] if c else oracle_mod.bfgs(p, x0)
        for k in KEYS:
            assert np.array_equal(g[k], o[k], equal_nan=True), (p.get("request_id"), k)


def test_required_c_full_size_d10(Z, ctx, oracle_mod):
    """The d = 10 Rastrigin workload at full size (N = 65,536) with early stop
    at 100 converged starts, every start against the oracle."""
    p = dict(W.RASTRIGIN_D10, required_converged=100)
    print("\n[required] rastrigin d10 full size, c = 100", flush=True)
    g = Z.zeus_minimize(ctx, p)
    o, kstar = oracle_mod.bfgs_required(W.RASTRIGIN_D10, oracle_mod.pso(p)["x"], 100)
    print(f"[required]   K* = {kstar}, stopped {int(np.sum(o['status'] == 2))}", flush=True)
    for k in KEYS:
        assert np.array_equal(g[k], o[k], equal_nan=True), k
