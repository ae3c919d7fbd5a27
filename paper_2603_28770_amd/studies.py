"""Effectiveness studies on synthetic runs.

* N_correct against the dimension of Rastrigin's function (Sec. V-A, the box
  plot of correct solutions per dimension): 10^5 particles, 5 swarm sweeps,
  each run stopped once 100 starts have converged (Alg. 10's required count).
* N_correct and the time to 100 convergences against the number of swarm
  sweeps for 5-dimensional Rastrigin and Rosenbrock (Sec. V-C).
* Clustering of the converged end points (the confidence measure proposed as
  future work in Sec. VI): the end points are grouped by their coordinates,
  and the size of the lowest group says how often the best candidate region
  was reached.

A start is correct when the Euclidean distance between its end point and the
global minimiser is below 0.5 (the paper's N_correct criterion).  Every run
goes through the C ABI (zeus_minimize); the arithmetic is the GPU path's.
"""
import time

import numpy as np

from . import workloads as W

# coordinate of the global minimiser, the same on every axis
XSTAR = {
    "rastrigin": 0.0,
    "ackley": 0.0,
    "rosenbrock": 1.0,
    "styblinski_tang": W.ST_XSTAR,
    "sphere": 0.0,
    "quartic": 0.0,
}

ST_CONVERGED = 1


def n_correct(x, objective, radius=0.5, mask=None):
    """Number of end points (rows of x) within Euclidean distance `radius`
    of the global minimiser; `mask` restricts the count to some rows."""
    x = np.asarray(x, dtype=np.float64)
    if x.size == 0:
        return 0
    dist = np.sqrt(((x - XSTAR[objective]) ** 2).sum(axis=1))
    ok = dist < radius
    if mask is not None:
        ok &= np.asarray(mask, dtype=bool)
    return int(ok.sum())


def cluster_minima(x, f, radius):
    """Group end points by coordinates: taken in order of increasing f (lower
    index first on ties), a point joins the first existing group whose leader
    (its first, lowest point) lies within `radius`, else it leads a new group.
    Points with a non-finite f are left out.  Returns the groups in leader
    order as dicts {leader, f, count} (leader is a row index of x)."""
    x = np.asarray(x, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    order = np.lexsort((np.arange(f.size), f))
    leaders, counts = [], []
    for i in order:
        if not np.isfinite(f[i]):
            continue
        if leaders:
            d = np.sqrt(((x[leaders] - x[i]) ** 2).sum(axis=1))
            hit = np.flatnonzero(d < radius)
            if hit.size:
                counts[hit[0]] += 1
                continue
        leaders.append(int(i))
        counts.append(1)
    return [{"leader": li, "f": float(f[li]), "count": c} for li, c in zip(leaders, counts)]


def run_summary(out, objective, radius=0.5):
    """Per-run figures from one zeus_minimize result dict."""
    conv = out["status"] == ST_CONVERGED
    xc = out["x"][conv]
    groups = cluster_minima(xc, out["f"][conv], radius)
    lowest = groups[0] if groups else None
    return {
        "n_correct": n_correct(out["x"], objective, radius),
        "n_correct_converged": n_correct(out["x"], objective, radius, conv),
        "n_converged": int(conv.sum()),
        "groups": len(groups),
        "lowest_group_count": lowest["count"] if lowest else 0,
        "lowest_group_correct": bool(lowest) and n_correct(xc[[lowest["leader"]]], objective, radius) == 1,
        "best_f": float(out["summary"]["best_f"]),
    }


def _quartiles(v):
    v = np.asarray(v, dtype=np.float64)
    q = np.percentile(v, [0, 25, 50, 75, 100])
    return {"min": q[0], "q1": q[1], "median": q[2], "q3": q[3], "max": q[4], "mean": float(v.mean())}


def study_problem(objective, dim, n, iter_pso, seed, required_c, iter_bfgs=1000):
    lo, hi = W.BOXES[objective]
    return W.problem(objective=objective, dim=dim, n=n, lower=lo, upper=hi, iter_pso=iter_pso,
                     iter_bfgs=iter_bfgs, seed=seed, required_converged=required_c)


def sweep(Z, ctx, objective, configs, runs, n, required_c, seed0, log=None):
    """configs: list of (dim, iter_pso).  For each, `runs` runs with seeds
    seed0, seed0 + 1, ...; returns one row per config with the quartiles of
    N_correct (all starts and converged starts), of the lowest group's size,
    of the wall time per run (blocking call, results copied to host) and of
    the device time of its kernels (swarm, every BFGS pass up to the required
    count of convergences, summary; HIP events on the context's stream)."""
    rows = []
    for dim, iter_pso in configs:
        per = []
        times, gpu = [], []
        for r in range(runs):
            p = study_problem(objective, dim, n, iter_pso, seed0 + r, required_c)
            Z.zeus_context_set_profiling(ctx, True)
            t0 = time.perf_counter()
            out = Z.zeus_minimize(ctx, p, ls_trials=False)
            times.append(time.perf_counter() - t0)
            pr = Z.zeus_context_get_profile(ctx)
            Z.zeus_context_set_profiling(ctx, False)
            gpu.append(pr["pso_ms"] + pr["bfgs_ms"] + pr["reduce_ms"])
            per.append(run_summary(out, objective))
        row = {
            "objective": objective, "dim": dim, "iter_pso": iter_pso, "runs": runs, "n": n,
            "required_converged": required_c,
            "n_correct": _quartiles([s["n_correct"] for s in per]),
            "n_correct_converged": _quartiles([s["n_correct_converged"] for s in per]),
            "lowest_group_count": _quartiles([s["lowest_group_count"] for s in per]),
            "lowest_group_correct_share": float(np.mean([s["lowest_group_correct"] for s in per])),
            "run_ms": _quartiles(np.array(times) * 1e3),
            "gpu_ms": _quartiles(gpu),
        }
        rows.append(row)
        if log:
            log(f"[study] {objective} d={dim} pso={iter_pso}: N_correct median "
                f"{row['n_correct']['median']:.0f}, run {row['run_ms']['median']:.2f} ms, "
                f"kernels {row['gpu_ms']['median']:.2f} ms")
    return rows
