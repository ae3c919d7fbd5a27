"""Plans (zeus_plan_*): a batch captured into a HIP graph and replayed.  Every
replay, with the program's own eager solves and synchronisations between the
replays, must equal the eager zeus_minimize results bit for bit."""
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


def _mix():
    return [
        W.scaled(W.RASTRIGIN_D10, 3000),
        W.problem(name="ros33", objective="rosenbrock", dim=33, n=300, lower=-3.0, upper=3.0,
                  iter_pso=3, iter_bfgs=400, seed=2),
        W.problem(name="st90", objective="styblinski_tang", dim=90, n=40, lower=-5.0, upper=5.0,
                  iter_pso=2, iter_bfgs=200, seed=7, precision="mixed", grad_tol=1e-4),
        W.problem(name="ack5", objective="ackley", dim=5, n=900, lower=-5.0, upper=5.0,
                  iter_pso=0, iter_bfgs=300, seed=9),
    ]


def test_plan_replays_equal_eager(Z, ctx):
    import torch
    reqs = _mix()
    eager = [Z.zeus_minimize(ctx, p) for p in reqs]
    plan = Z.DevicePlan(ctx, reqs, trace_len=4)
    stream = torch.cuda.Stream()
    for rep in range(4):
        print(f"\n[plan] replay {rep}", flush=True)
        plan.launch(stream.cuda_stream)
        torch.cuda.synchronize()
        got = plan.host()
        for r, (a, b) in enumerate(zip(eager, got)):
            for k in KEYS:
                assert np.array_equal(a[k], b[k], equal_nan=True), (rep, r, k)
            assert a["summary"] == b["summary"], (rep, r)
        # the program's own eager work between replays
        Z.zeus_minimize(ctx, W.scaled(W.ROSENBROCK_D2, 64 + rep))
    plan.close()


def test_plan_rejects_swarm_outputs(Z, ctx):
    """Swarm-state outputs need copies, which plans do not capture: refused
    before anything is enqueued (a real workspace is passed all the same)."""
    import ctypes as C
    import torch
    p = Z.make_problem(W.scaled(W.ROSENBROCK_D2, 32))
    wb = C.c_size_t()
    assert Z.lib.zeus_plan_workspace_bytes(C.byref(p), 1, C.byref(wb)) == Z.OK
    assert wb.value > 0
    ws = torch.empty(wb.value + 256, dtype=torch.uint8, device="cuda")
    ws_ptr = (ws.data_ptr() + 255) // 256 * 256
    dev = {k: torch.empty(32 * 2, dtype=torch.float64, device="cuda") for k in ("f", "x", "seeds")}
    ints = {k: torch.empty(32, dtype=torch.int32, device="cuda") for k in ("iters", "status")}
    summ = torch.empty(C.sizeof(Z.zeus_summary), dtype=torch.uint8, device="cuda")
    r = Z.zeus_result(f=dev["f"].data_ptr(), x=dev["x"].data_ptr(), iters=ints["iters"].data_ptr(),
                      status=ints["status"].data_ptr(), seeds=dev["seeds"].data_ptr(),
                      summary=summ.data_ptr())
    h = C.c_void_p()
    code = Z.lib.zeus_plan_create(ctx, C.byref(p), 1, C.c_void_p(ws_ptr), wb, C.byref(r), C.byref(h))
    assert code == Z.EINVAL and not h.value
