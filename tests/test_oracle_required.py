"""The oracle's early stop (Alg. 10 with required_c), checked against its
definition recomputed from the full run: K* is the required_c-th smallest
convergence iteration; starts that ended by K* keep the full run's results;
every other start stops at K* with its K*-th iterate, which a separate run
with a budget of K* iterations reproduces."""
import numpy as np

from paper_2603_28770_amd import workloads as W


def _p(**kw):
    base = dict(objective="rastrigin", dim=4, n=300, lower=-5.12, upper=5.12, iter_pso=3,
                iter_bfgs=200, seed=8)
    base.update(kw)
    return W.problem(**base)


def test_required_c_matches_its_definition(oracle_any):
    O = oracle_any
    p = _p()
    x0 = O.pso(p)["x"]
    full = O.bfgs(p, x0)
    conv_it = np.sort(full["iters"][full["status"] == 1])
    c = 37
    assert conv_it.size >= c
    r, kstar = O.bfgs_required(p, x0, c)
    assert kstar == conv_it[c - 1]
    early = full["iters"] <= kstar
    for k in ("x", "f", "iters", "status", "ls_trials"):
        assert np.array_equal(r[k][early], full[k][early])
    late = ~early
    assert np.all(r["status"][late] == 2) and np.all(r["iters"][late] == kstar)
    # the stopped iterates are the trajectories' K*-th points
    tr = O.bfgs(p, x0, trace_len=kstar + 1)["trace"]
    assert np.array_equal(r["x"][late], tr[late, kstar])
    assert np.sum(r["status"] == 1) >= c
    assert np.all(r["iters"] <= kstar)


def test_required_c_edge_cases(oracle_any):
    O = oracle_any
    p = _p(n=120)
    x0 = O.pso(p)["x"]
    full = O.bfgs(p, x0)
    nconv = int(np.sum(full["status"] == 1))
    # more than can converge: nothing stops
    r, kstar = O.bfgs_required(p, x0, nconv + 1)
    assert kstar is None and np.array_equal(r["status"], full["status"])
    # one convergence: K* is the fastest start's iteration count
    r, kstar = O.bfgs_required(p, x0, 1)
    assert kstar == full["iters"][full["status"] == 1].min()
    assert np.sum(r["status"] == 1) >= 1 and np.all(r["iters"] <= kstar)
