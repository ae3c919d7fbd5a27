"""The serving path (zeus_server_*) on the GPU: requests submitted from
several threads while others run come back bit-identical to solving each
alone; a short request that arrives during a long one is admitted at once,
shares the long one's steps on the device and ends first, with the same
results as alone; admission by device-memory footprint; cancel, poll and
shutdown."""
import threading
import time

import numpy as np
import pytest

from paper_2603_28770_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("f", "x", "iters", "status", "ls_trials", "skips", "resets", "seeds")


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


def _requests(count, seed, dmax=200, nmin=64, nspan=8.0):
    g = np.random.Generator(np.random.Philox(key=seed))
    u = g.random((count, 5))
    out = []
    for r in range(count):
        obj = W.MIX[min(int(u[r, 0] * 4), 3)]
        d = 2 + int(u[r, 1] * (dmax - 1))
        lo, hi = W.BOXES[obj]
        mixed = u[r, 4] < 0.5
        out.append(W.problem(name=f"s{r}", objective=obj, dim=d, n=int(nmin * nspan ** u[r, 2]),
                             lower=lo, upper=hi, iter_pso=int(u[r, 3] * 11), iter_bfgs=200,
                             seed=seed, request_id=r, precision="mixed" if mixed else "fp64",
                             grad_tol=1e-4 if mixed else 1e-6))
    return out


def _same(a, b):
    for k in KEYS:
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    assert a["summary"] == b["summary"]


def test_served_from_threads_equals_alone(Z, ctx):
    reqs = _requests(24, 31)
    print(f"\n[server] {len(reqs)} requests, d {min(p['dim'] for p in reqs)}.."
          f"{max(p['dim'] for p in reqs)}", flush=True)
    got = {}
    with Z.Server(ctx, 8 << 30) as srv:
        tickets = {}
        lock = threading.Lock()

        def client(part):
            for r in part:
                t = srv.submit(reqs[r], pso_state=True)
                with lock:
                    tickets[r] = t
                time.sleep(0.002 * (r % 3))

        th = [threading.Thread(target=client, args=(list(range(k, len(reqs), 3)),)) for k in range(3)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        for r, t in tickets.items():
            got[r] = srv.wait(t, timeout_s=120)
    for r, p in enumerate(reqs):
        a = Z.zeus_minimize(ctx, p, pso_state=True)
        _same(a, got[r])
        tm = got[r]["times"]
        assert tm["t_submit_ns"] <= tm["t_admit_ns"] <= tm["t_done_ns"]


def test_tight_budget_queues_and_rejects(Z, ctx):
    reqs = _requests(8, 7, dmax=60, nmin=256, nspan=4.0)
    need = [Z.Server.request_bytes(p) for p in reqs]
    # requests get three quarters of the budget: room for one or two at a time
    budget = (max(need) * 2 + (1 << 20)) * 4 // 3
    with Z.Server(ctx, budget) as srv:
        tickets = [srv.submit(p) for p in reqs]
        outs = [srv.wait(t, timeout_s=120) for t in tickets]
        big = W.problem(objective="sphere", dim=256, n=1 << 20, lower=-1.0, upper=1.0)
        with pytest.raises(Z.ZeusError) as e:
            srv.submit(big)
        assert e.value.code == Z.ENOMEM
    admits = sorted(o["times"]["t_admit_ns"] for o in outs)
    assert admits[-1] > admits[0]  # not all admitted at once
    for p, o in zip(reqs, outs):
        a = Z.zeus_minimize(ctx, p)
        for k in ("f", "x", "iters", "status"):
            assert np.array_equal(a[k], o[k], equal_nan=True)


def test_cancel_poll_and_shutdown(Z, ctx):
    long = W.problem(objective="rosenbrock", dim=50, n=20000, lower=-5.0, upper=5.0, iter_pso=2,
                     iter_bfgs=2000, seed=3)
    small = W.problem(objective="sphere", dim=4, n=64, lower=-1.0, upper=1.0, seed=4)
    srv = Z.Server(ctx, 4 << 30)
    t1 = srv.submit(long)
    ts = [srv.submit(dict(small, request_id=k)) for k in range(6)]
    code = srv.cancel(ts[-1])
    if code == Z.OK:
        with pytest.raises(Z.ZeusError) as e:
            srv.wait(ts[-1], timeout_s=60)
        assert e.value.code == Z.ECANCELLED
    else:
        assert code == Z.NOT_READY and srv.wait(ts[-1], timeout_s=60) is not None
    polled = srv.wait(t1, timeout_s=0)   # None while it runs
    res = polled if polled is not None else srv.wait(t1, timeout_s=120)
    assert res["summary"]["n_converged"] > 0
    with pytest.raises(Z.ZeusError) as e:
        srv.wait(t1, timeout_s=0)   # released
    assert e.value.code == Z.EINVAL
    # leave tickets unwaited: destroy cancels what is queued and drains the rest
    for k in range(3):
        srv.submit(dict(small, request_id=100 + k))
    srv.close()


def test_short_request_during_long(Z, ctx):
    """Continuous batching at the level of starts: a long request (the d = 50
    Rosenbrock problem with all its 131,072 starts, many steps, about 60 ms of
    BFGS) is running when a short one of the same kernel class arrives 5 ms
    later; the short one is admitted at once, takes a share of the next steps
    beside the long one, ends long before it, and both equal their solves
    alone bit for bit."""
    long_ = dict(W.ROSENBROCK_D50, request_id=1)
    short = dict(W.ROSENBROCK_D50, n=512, request_id=2)
    a_long, a_short = Z.zeus_minimize(ctx, long_), Z.zeus_minimize(ctx, short)
    with Z.Server(ctx, 8 << 30) as srv:
        t_long = srv.submit(long_)
        time.sleep(0.005)
        t_short = srv.submit(short)
        o_short = srv.wait(t_short, timeout_s=120)
        o_long = srv.wait(t_long, timeout_s=120)
    s, l = o_short["times"], o_long["times"]
    print(f"\n[server] long admitted..done {(l['t_done_ns'] - l['t_admit_ns']) / 1e6:.1f} ms; "
          f"short submitted {(s['t_submit_ns'] - l['t_admit_ns']) / 1e6:.1f} ms after it, "
          f"done after {(s['t_done_ns'] - s['t_submit_ns']) / 1e6:.1f} ms", flush=True)
    assert l["t_admit_ns"] < s["t_submit_ns"] and s["t_admit_ns"] < l["t_done_ns"]
    assert s["t_done_ns"] < l["t_done_ns"]
    _same_keys = ("f", "x", "iters", "status", "ls_trials", "skips", "resets")
    for a, o in ((a_long, o_long), (a_short, o_short)):
        for k in _same_keys:
            assert np.array_equal(a[k], o[k], equal_nan=True), k
        assert a["summary"] == o["summary"]
