"""The default build's readings (balanced pairwise sums, blocked fused row
products, the two-FMA update, Cody-Waite sin/cos/exp) against the plain build
(textbook order, the C library's functions), at the stated tolerances of
tests/plain_check.py: the readings fix the order of rounding but change no
result beyond them.  CPU only; reduced start counts of the benchmark
workloads."""
import numpy as np
import pytest

from paper_2603_28770_amd import workloads as W
from tests import plain_check as PC

CASES = [
    (W.ROSENBROCK_D2, None),
    (W.scaled(W.RASTRIGIN_D10, 4096), 256),
    (W.scaled(W.ROSENBROCK_D50, 2048), 32),
    (W.scaled(W.ACKLEY_D50, 2048), 32),
]


def _default_solve(O, p, sample):
    idx = None if sample is None else W.strided_subset(p["n"], sample)
    sw = O.pso(p)
    r = O.bfgs(p, sw["x"], idx=idx, trace_len=PC.L)
    n, d = p["n"], p["dim"]
    sel = np.arange(n) if idx is None else idx
    g = {"seeds": sw["x"], "pso_pf": sw["pf"], "summary": {"pso_best_index": sw["gidx"]},
         "f": np.full(n, np.nan), "iters": np.full(n, -1, np.int32),
         "status": np.full(n, -1, np.int32), "trace": np.full((n, PC.L, d), np.nan)}
    for k in ("f", "iters", "status", "trace"):
        g[k][sel] = r[k]
    return g


@pytest.mark.parametrize("p,sample", CASES, ids=[c[0]["name"] for c in CASES])
def test_default_readings_within_tolerance_of_plain(oracle_mod, p, sample):
    PC.check_against_plain(_default_solve(oracle_mod, p, sample), p, sample)
