"""Pins for the oracle's swarm (Sec. III-A, Alg. 2 and Alg. 3, read
synchronously): the initial swarm is an affine map of the pinned uniform
stream, degenerate coefficients reduce the update to straight lines and
geometric velocities, personal bests never get worse and the global best is
always the first minimum of the personal bests."""
import numpy as np
import pytest

from paper_2603_28770_amd.workloads import problem

M256 = (1 << 256) - 1


def _u(seed, req, i, t, tag, j):
    # independent route to the same uniform: numpy's Philox + Generator.random
    c = (j // 4) | (i << 64) | (t << 128) | (tag << 192)
    g = np.random.Generator(np.random.Philox(counter=(c - 1) & M256, key=seed | (req << 64)))
    return g.random(j % 4 + 1)[-1]


@pytest.mark.parametrize("obj,d,lo,hi,vh", [("rosenbrock", 2, -5.0, 5.0, 1.0),
                                           ("rastrigin", 5, -5.12, 5.12, 0.0),
                                           ("styblinski_tang", 3, -5.0, 5.0, 0.0)])
def test_initial_swarm_is_affine_map_of_stream(oracle_any, obj, d, lo, hi, vh):
    p = problem(objective=obj, dim=d, n=37, lower=lo, upper=hi, v_half=vh, seed=9, request_id=4)
    sw = oracle_any.pso(p)
    V = vh if vh > 0 else hi - lo
    for i in range(p["n"]):
        for j in range(d):
            ux, uv = _u(9, 4, i, 0, 0, j), _u(9, 4, i, 0, 1, j)
            assert sw["x"][i, j] == lo + ux * (hi - lo)
            assert sw["v"][i, j] == -V + uv * (V - (-V))
            assert lo <= sw["x"][i, j] <= hi and -V <= sw["v"][i, j] <= V
    assert np.array_equal(sw["px"], sw["x"])
    assert all(sw["pf"][i] == oracle_any.f(obj, sw["x"][i]) for i in range(p["n"]))
    g = int(np.argmin(sw["pf"]))           # numpy: first index of the minimum
    assert sw["gidx"] == g and sw["gf"] == sw["pf"][g] and np.array_equal(sw["gx"], sw["x"][g])


def test_pure_inertia_is_a_straight_line(oracle_any):
    # w = 1, c1 = c2 = 0: v stays v0 and x_t = x_{t-1} + v0
    base = problem(objective="sphere", dim=3, n=16, lower=-1.0, upper=1.0, w=1.0, c1=0.0, c2=0.0)
    s0 = oracle_any.pso(dict(base, iter_pso=0))
    sT = oracle_any.pso(dict(base, iter_pso=6))
    x = s0["x"].copy()
    for _ in range(6):
        x = x + s0["v"]
    assert np.array_equal(sT["x"], x) and np.array_equal(sT["v"], s0["v"])


def test_half_inertia_geometric_velocity(oracle_any):
    # w = 0.5, c1 = c2 = 0: v_t = v0 / 2^t exactly
    base = problem(objective="rastrigin", dim=4, n=8, lower=-2.0, upper=2.0, w=0.5, c1=0.0, c2=0.0)
    s0 = oracle_any.pso(dict(base, iter_pso=0))
    sT = oracle_any.pso(dict(base, iter_pso=5))
    assert np.array_equal(sT["v"], s0["v"] / 32.0)


def test_cognitive_only_step(oracle_any):
    # w = 0, c2 = 0, one step: v = (c1 r1)(p - x) with p = x at t = 0 -> v = 0, x unchanged
    base = problem(objective="rosenbrock", dim=2, n=8, lower=-2.0, upper=2.0, w=0.0, c1=1.3, c2=0.0)
    s0 = oracle_any.pso(dict(base, iter_pso=0))
    s1 = oracle_any.pso(dict(base, iter_pso=1))
    assert np.array_equal(s1["x"], s0["x"]) and np.all(s1["v"] == 0.0)


def test_social_only_first_step_moves_toward_initial_best(oracle_any):
    # w = 0, c1 = 0, c2 = 1: x_1 = x_0 + r2 (g_0 - x_0), a point of the segment [x_0, g_0]
    base = problem(objective="sphere", dim=3, n=32, lower=-4.0, upper=4.0, w=0.0, c1=0.0, c2=1.0,
                   seed=5)
    s0 = oracle_any.pso(dict(base, iter_pso=0))
    s1 = oracle_any.pso(dict(base, iter_pso=1))
    for i in range(32):
        for j in range(3):
            r2 = _u(5, 0, i, 1, 3, j)
            x0, g0 = s0["x"][i, j], s0["gx"][j]
            assert s1["x"][i, j] == x0 + (1.0 * r2) * (g0 - x0)
    # the particle that is the global best does not move
    g = s0["gidx"]
    assert np.array_equal(s1["x"][g], s0["x"][g])


@pytest.mark.parametrize("obj,d", [("rastrigin", 3), ("rosenbrock", 4), ("ackley", 5)])
def test_bests_monotone_and_consistent(oracle_any, obj, d):
    base = problem(objective=obj, dim=d, n=200, lower=-5.0, upper=5.0, seed=21)
    prev = None
    for t in range(0, 8):
        sw = oracle_any.pso(dict(base, iter_pso=t))
        for i in range(base["n"]):
            assert sw["pf"][i] == oracle_any.f(obj, sw["px"][i])
        g = int(np.argmin(sw["pf"]))
        assert sw["gf"] == sw["pf"][g] and sw["gidx"] == g and np.array_equal(sw["gx"], sw["px"][g])
        if prev is not None:
            assert np.all(sw["pf"] <= prev["pf"])
            assert sw["gf"] <= prev["gf"]
        prev = sw


def test_global_best_ties_take_lowest_index(oracle_any):
    # sphere over a box symmetric in sign with w = c1 = c2 = 0: nobody moves and
    # particles whose coordinates are negatives of each other tie exactly; the
    # global best must still be the first index attaining the minimum value
    sw = oracle_any.pso(problem(objective="sphere", dim=1, n=4096, lower=-1.0, upper=1.0,
                                iter_pso=2, w=0.0, c1=0.0, c2=0.0, seed=2))
    m = sw["pf"].min()
    assert sw["gidx"] == int(np.flatnonzero(sw["pf"] == m)[0])
