"""The comparison of a solve against the plain build of the oracle at the
stated tolerances (shared by the GPU test and the CPU test of the default
build's readings).  See tests/test_gpu_plain_oracle.py for the bars."""
import numpy as np

from paper_2603_28770_amd import workloads as W

TRAJ_TOL = 1e-9
F_TOL = 1e-6
L = 20


def check_against_plain(g, p, sample, min_within=0.85, min_same=0.99):
    """g: a solve of problem p with its swarm state and the first L iterates
    (keys seeds, pso_pf, f, iters, status, trace, summary.pso_best_index).
    Compares the whole swarm and the starts of a strided sample of `sample`
    starts (all when None) with the plain oracle; returns the figures."""
    from oracle import oracle as O
    idx = None if sample is None else W.strided_subset(p["n"], sample)
    sw = O.pso(p, plain=True)
    o = O.bfgs(p, sw["x"], idx=idx, trace_len=L, plain=True)
    sel = np.arange(p["n"]) if idx is None else idx

    # swarm
    assert g["summary"]["pso_best_index"] == sw["gidx"]
    same_seed = np.all(g["seeds"] == sw["x"], axis=1)
    dpf = np.abs(g["pso_pf"] - sw["pf"]) / np.maximum(1.0, np.abs(sw["pf"]))
    print(f"[plain]   swarm: identical positions {same_seed.mean():.5f}, "
          f"personal-best values max rel diff {dpf[same_seed].max():.2e}", flush=True)
    assert same_seed.mean() >= 0.999
    assert dpf[same_seed].max() <= 1e-12

    # trajectories of the starts whose seeds are identical
    ok = same_seed[sel]
    tg, to = g["trace"][sel][ok], o["trace"][ok]
    with np.errstate(invalid="ignore"):
        scale = np.maximum(1.0, np.nanmax(np.abs(to), axis=2, initial=0.0))
        err = np.nanmax(np.abs(tg - to), axis=2, initial=0.0) / scale
    # iterates both sides reached (a start may converge one step earlier on
    # one side: the test ||g|| < Theta is then a near-tie; its final result is
    # checked below)
    both = np.isfinite(tg).all(axis=2) & np.isfinite(to).all(axis=2)
    # iterates up to the oracle's first near-tie decision (a branch whose
    # relative margin was below 1e-9: an Armijo test at the noise level of f
    # next to a minimum, where either rounding may take the other branch)
    tie = o["tie_iter"][ok]
    upto = np.where(tie >= 0, tie, L)[:, None] >= np.arange(L)[None, :]
    err = np.where(both & upto, err, 0.0)
    worst = err.max(axis=0)
    print("[plain]   worst iterate drift per step: " +
          " ".join(f"{k}:{worst[k]:.1e}" for k in (0, 1, 2, 3, 5, 10, 15, 19)), flush=True)
    within = np.all(err <= TRAJ_TOL, axis=1)
    print(f"[plain]   starts within {TRAJ_TOL:g} over all {L} iterates: {within.mean():.4f}",
          flush=True)
    assert np.all(err[:, :6] <= TRAJ_TOL)
    assert within.mean() >= min_within

    # final results
    gf, gs = g["f"][sel], g["status"][sel]
    fs = np.maximum(1.0, np.abs(o["f"]))
    with np.errstate(invalid="ignore"):
        df = np.where((gf == o["f"]) | (~np.isfinite(gf) & ~np.isfinite(o["f"])), 0.0,
                      np.abs(gf - o["f"]) / fs)
    same = (gs == o["status"]) & (df <= F_TOL)
    fstar = W.f_star(p["objective"], p["dim"])
    rg, ro = np.mean(gf - fstar < 1e-4), np.mean(o["f"] - fstar < 1e-4)
    print(f"[plain]   same status and f within {F_TOL:g}: {same.mean():.4f}; |df| max "
          f"{np.nanmax(df):.2e}; same iteration count {np.mean(g['iters'][sel] == o['iters']):.4f}; "
          f"success {rg:.4f} plain oracle {ro:.4f}", flush=True)
    assert same.mean() >= min_same
    assert abs(rg - ro) <= 0.01
    return {"within": float(within.mean()), "same": float(same.mean()),
            "worst": worst.tolist()}
