"""The server's scheduling on the emulated device (no GPU): admission by
memory in arrival order, the sharing of steps between requests, queueing,
cancellation, shutdown and submissions from several threads.  On the emulated
device a swarm, a step and a finish take modelled host time and the results
are placeholders (f = request id), so these tests see only the scheduling."""
import threading
import time

import numpy as np
import pytest

from paper_2603_28770_amd import workloads as W

MS = 1_000_000  # ns


@pytest.fixture(scope="module")
def Z():
    from paper_2603_28770_amd import zeus
    return zeus


def req(n, rid, d=10):
    return W.problem(name=f"r{rid}", objective="rastrigin", dim=d, n=n, lower=-5.12, upper=5.12,
                     iter_pso=2, iter_bfgs=50, request_id=rid)


def server(Z, budget, **emu):
    kw = dict(swarm_ns=1 * MS, step_ns=1 * MS, start_ns=2 * MS, finish_ns=0, resident_starts=512)
    kw.update(emu)
    return Z.Server.emulated(budget, **kw)


def arena(budget):
    """Bytes of the step buffers: min(budget / 4, 2 GiB), in whole 512-byte units."""
    return min(budget // 4, 2 << 30) // 512 * 512


def test_request_bytes_counts_the_asked_outputs(Z):
    p = req(4096, 0)
    base = Z.Server.request_bytes(p)
    with_state = Z.Server.request_bytes(p, pso_state=True)
    # x, v, px of the swarm as outputs: 3 N d doubles more (256-byte pieces)
    assert with_state - base >= 3 * 4096 * 10 * 8
    assert Z.Server.request_bytes(dict(p, required_converged=5)) > base


def test_admission_in_order_within_budget(Z):
    """At no time do the admitted requests hold more than the budget, and they
    are admitted in arrival order."""
    p = req(2048, 0)
    one = Z.Server.request_bytes(p)
    budget = 4 * (2 * one + one // 2) // 3 + 4096  # requests' share: two and a half
    assert budget - arena(budget) >= 2 * one and budget - arena(budget) < 3 * one
    with server(Z, budget) as srv:
        ts = [srv.submit(dict(p, request_id=r)) for r in range(6)]
        outs = [srv.wait(t, timeout_s=30) for t in ts]
    iv = [(o["times"]["t_admit_ns"], o["times"]["t_done_ns"]) for o in outs]
    assert [a for a, _ in iv] == sorted(a for a, _ in iv)
    for a, _ in iv:
        held = sum(1 for a2, d2 in iv if a2 <= a < d2)
        assert held <= 2
    for r, o in enumerate(outs):
        assert np.all(o["f"] == r) and o["summary"]["best_f"] == r


def test_short_request_finishes_inside_a_long_one(Z):
    """A short request that arrives while a long one is running is admitted at
    once, shares the next step, and ends long before the long one."""
    with server(Z, 1 << 30) as srv:
        t_long = srv.submit(req(64 * 512, 1))   # 16 steps of 4 resident rounds
        time.sleep(0.01)
        t_short = srv.submit(req(256, 2))
        short = srv.wait(t_short, timeout_s=30)
        long_ = srv.wait(t_long, timeout_s=60)
    s, l = short["times"], long_["times"]
    assert s["t_admit_ns"] < l["t_done_ns"] and s["t_done_ns"] < l["t_done_ns"]
    # the short request waits for at most a few steps, not for the long one
    assert s["t_done_ns"] - s["t_submit_ns"] < (l["t_done_ns"] - l["t_admit_ns"]) / 3


def test_equal_requests_share_the_steps(Z):
    """Two equal requests admitted together progress together (each step gives
    both an equal slice), so they end close together rather than one after
    the other.  Run one after the other, the first would end halfway through
    the span; the bound leaves room for the steps built before the second's
    swarm ended and for a scheduling thread slowed by a loaded host (the
    emulated device's operations are host time)."""
    with server(Z, 1 << 30) as srv:
        ts = [srv.submit(req(64 * 512, r)) for r in (1, 2)]
        outs = [srv.wait(t, timeout_s=60) for t in ts]
    d = [o["times"]["t_done_ns"] for o in outs]
    span = max(d) - min(o["times"]["t_admit_ns"] for o in outs)
    assert abs(d[0] - d[1]) < 0.3 * span


def test_cancel_queued_and_running(Z):
    p = req(8 * 512, 0)
    one = Z.Server.request_bytes(p)
    budget = 4 * (one + one // 2) // 3 + 4096  # room for one request at a time
    with server(Z, budget) as srv:
        a = srv.submit(dict(p, request_id=1))
        b = srv.submit(dict(p, request_id=2))
        c = srv.submit(dict(p, request_id=3))
        time.sleep(0.005)
        assert srv.cancel(a) == Z.NOT_READY        # admitted: runs to its end
        assert srv.cancel(b) == Z.OK               # queued: never runs
        with pytest.raises(Z.ZeusError) as e:
            srv.wait(b, timeout_s=1)
        assert e.value.code == Z.ECANCELLED
        oa, oc = srv.wait(a, timeout_s=30), srv.wait(c, timeout_s=30)
        assert np.all(oa["f"] == 1) and np.all(oc["f"] == 3)
        assert oc["times"]["t_admit_ns"] >= oa["times"]["t_done_ns"]
        with pytest.raises(Z.ZeusError) as e:
            srv.wait(b, timeout_s=0)               # released
        assert e.value.code == Z.EINVAL


def test_poll_timeout_and_too_large(Z):
    with server(Z, 64 << 20, start_ns=20 * MS) as srv:
        t = srv.submit(req(4096, 5))
        assert srv.wait(t, timeout_s=0) is None    # still running
        with pytest.raises(Z.ZeusError) as e:
            srv.wait(t, timeout_s=0.001)
        assert e.value.code == Z.ETIMEOUT
        assert np.all(srv.wait(t, timeout_s=30)["f"] == 5)
        with pytest.raises(Z.ZeusError) as e:
            srv.submit(req(1 << 20, 6))            # about 200 MB of state
        assert e.value.code == Z.ENOMEM


def test_shutdown_cancels_the_queue_and_drains_the_running(Z):
    p = req(8 * 512, 0)
    one = Z.Server.request_bytes(p)
    budget = 4 * (one + one // 2) // 3 + 4096
    srv = server(Z, budget)
    srv.submit(dict(p, request_id=7))
    srv.submit(dict(p, request_id=8))
    time.sleep(0.005)
    first, second = [srv._live[t][1] for t in sorted(srv._live)]
    srv.close()                                    # waits for the admitted one
    assert np.all(first["f"] == 7)
    assert np.all(np.isnan(second["f"]))           # never ran


def test_submissions_from_threads(Z):
    with server(Z, 1 << 30, swarm_ns=MS // 10, step_ns=MS // 10, start_ns=MS // 5) as srv:
        got = {}
        lock = threading.Lock()

        def client(k):
            for i in range(8):
                rid = 100 * k + i
                o = srv.wait(srv.submit(req(300 + 37 * i, rid, d=2 + i)), timeout_s=60)
                with lock:
                    got[rid] = o

        th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
    assert len(got) == 32
    for rid, o in got.items():
        assert np.all(o["f"] == rid)
