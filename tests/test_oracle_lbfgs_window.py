"""Pins for the oracle's L-BFGS pair window (the history of (s, y) pairs the
two-loop recursion reads; Nocedal and Wright, "Numerical Optimization", 2nd
ed., Sec. 7.2, the remedy the paper names for the cost of the full inverse-
Hessian update).  The window holds the newest m pairs with y's > 0, oldest
first; a pair with y's <= 0 is skipped; a restart from H = I empties it.

Two kinds of pin:
  * the window update itself (zo_lbfgs_push) on hand-made pairs;
  * a replay of whole oracle trajectories: from the traced iterates x_k the
    test rebuilds g_k (zo_grad), s_k and y_k, keeps its own window by the
    rule above, and requires every step to be x_{k+1} = x_k + alpha p_k with
    p_k the two-loop direction over that window and alpha = shrink^j for
    some j <= iter_ls, bit for bit.  Replays under the plausible mistakes
    (keeping the oldest m pairs, keeping m + 1, keeping pairs with y's <= 0)
    must fail on the same trajectories, which shows that the replay sees
    them.

The restart branch (g'p not < 0) empties the window.  With every stored pair
of positive curvature the two-loop direction is a descent direction in exact
arithmetic, and no trajectory of these objectives reaches the branch (the
replay asserts zero restarts), so that part of the rule is pinned only by the
window unit test of an empty window."""
import numpy as np
import pytest

from paper_2603_28770_amd import workloads as W


def test_push_keeps_newest_m_oldest_first(oracle_any):
    O = oracle_any
    d, m = 3, 4
    S, Y, rho = np.zeros((m, d)), np.zeros((m, d)), np.zeros(m)
    cnt = 0
    pairs = []
    for k in range(7):
        s = np.array([1.0 + k, 0.5, -0.25 * k])
        y = np.array([2.0, 1.0 + k, 0.0])
        cnt, ok = O.lbfgs_push(S, Y, rho, cnt, s, y)
        assert ok
        pairs.append((s, y))
        keep = pairs[-m:]
        assert cnt == len(keep)
        for i, (ss, yy) in enumerate(keep):
            assert np.array_equal(S[i], ss) and np.array_equal(Y[i], yy)
            assert rho[i] == 1.0 / float(np.dot(yy, ss))


def test_push_skips_non_positive_curvature(oracle_any):
    O = oracle_any
    S, Y, rho = np.zeros((2, 2)), np.zeros((2, 2)), np.zeros(2)
    cnt, ok = O.lbfgs_push(S, Y, rho, 0, [1.0, 0.0], [1.0, 5.0])
    assert ok and cnt == 1
    before = (S.copy(), Y.copy(), rho.copy())
    for y in ([-1.0, 0.0], [0.0, 1.0], [np.nan, 0.0]):   # y's < 0, = 0, NaN
        cnt2, ok2 = O.lbfgs_push(S, Y, rho, cnt, [1.0, 0.0], y)
        assert not ok2 and cnt2 == cnt
        assert all(np.array_equal(a, b) for a, b in zip(before, (S, Y, rho)))


def test_empty_window_is_steepest_descent(oracle_any):
    # what a restart leaves: no pairs, p = -g
    g = np.array([0.3, -2.0, 7.5])
    assert np.array_equal(oracle_any.lbfgs_direction(np.zeros((0, 3)), np.zeros((0, 3)),
                                                     np.zeros(0), g), -g)


def _replay(O, p, x_trace, rule="newest"):
    """Checks each traced step against the window rule; returns the number of
    steps reproduced before the first mismatch and the number checked."""
    m, d = p["lbfgs_m"], p["dim"]
    ks = [k for k in range(x_trace.shape[0]) if np.all(np.isfinite(x_trace[k]))]
    xs = x_trace[: len(ks)]
    gs = [O.grad(p["objective"], x)[1] for x in xs]
    pairs = []
    for k in range(len(xs) - 1):
        if rule == "oldest":
            win = pairs[:m]
        elif rule == "m_plus_1":
            win = pairs[-(m + 1):]
        else:
            win = pairs[-m:]
        if win:
            S = np.array([a for a, _ in win])
            Y = np.array([b for _, b in win])
            rho = np.array([1.0 / O_dot(O, b, a) for a, b in win])
        else:
            S = Y = np.zeros((0, d))
            rho = np.zeros(0)
        dirn = O.lbfgs_direction(S, Y, rho, gs[k])
        if not float(np.dot(gs[k], dirn)) < 0:   # sign only
            # the oracle would restart here; the correct rule never gets here
            assert rule != "newest", "a restart was reached; the replay does not model it"
            return k, len(xs) - 1
        alpha, hit = 1.0, False
        for _ in range(p["iter_ls"] + 1):
            if np.array_equal(xs[k] + alpha * dirn, xs[k + 1]):
                hit = True
                break
            alpha *= p["ls_shrink"]
        if not hit:
            return k, len(xs) - 1
        s = xs[k + 1] - xs[k]
        y = gs[k + 1] - gs[k]
        if rule == "keep_negative" or O_dot(O, y, s) > 0:
            pairs.append((s, y))
    return len(xs) - 1, len(xs) - 1


def O_dot(O, a, b):
    # y's through the oracle's own window test: a one-pair push reports it
    S, Y, rho = np.zeros((1, a.size)), np.zeros((1, a.size)), np.zeros(1)
    _, ok = O.lbfgs_push(S, Y, rho, 0, b, a)
    return 1.0 / rho[0] if ok else -1.0


CASES = [
    W.problem(objective="rosenbrock", dim=6, n=24, lower=-2.0, upper=2.0, iter_pso=0,
              iter_bfgs=60, seed=3, lbfgs_m=3),
    W.problem(objective="rastrigin", dim=4, n=24, lower=-5.12, upper=5.12, iter_pso=0,
              iter_bfgs=60, seed=4, lbfgs_m=2),
    W.problem(objective="styblinski_tang", dim=5, n=24, lower=-5.0, upper=5.0, iter_pso=0,
              iter_bfgs=60, seed=5, lbfgs_m=5),
    W.problem(objective="ackley", dim=3, n=24, lower=-3.0, upper=3.0, iter_pso=0,
              iter_bfgs=60, seed=6, lbfgs_m=1),
    W.problem(objective="rosenbrock", dim=9, n=16, lower=-2.0, upper=2.0, iter_pso=0,
              iter_bfgs=80, seed=7, lbfgs_m=8),
]


@pytest.mark.parametrize("p", CASES, ids=lambda p: f"{p['objective']}_d{p['dim']}_m{p['lbfgs_m']}")
def test_trajectories_follow_the_window_rule(oracle_any, p):
    O = oracle_any
    L = p["iter_bfgs"] + 1
    r = O.bfgs(p, O.pso(p)["x"], trace_len=L)
    assert r["resets"].sum() == 0
    checked = 0
    for s in range(p["n"]):
        done, total = _replay(O, p, r["trace"][s])
        assert done == total, (s, done, total)
        checked += total
    assert checked > 100


def test_replay_sees_window_mistakes(oracle_any):
    """Each mistaken rule fails to reproduce some step of these trajectories."""
    O = oracle_any
    caught = {"oldest": 0, "m_plus_1": 0, "keep_negative": 0}
    skips = 0
    for p in CASES:
        r = O.bfgs(p, O.pso(p)["x"], trace_len=p["iter_bfgs"] + 1)
        skips += int(r["skips"].sum())
        for s in range(p["n"]):
            for rule in caught:
                done, total = _replay(O, p, r["trace"][s], rule)
                caught[rule] += done < total
    assert skips > 0, "no pair with y's <= 0 in these trajectories"
    assert all(v > 0 for v in caught.values()), caught
