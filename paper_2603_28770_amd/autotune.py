"""Tiling autotuner for the BFGS kernels (run on the target GPU).

    python -m paper_2603_28770_amd.autotune [--quick] [--out PATH]

For every objective, precision and probe dimension it times each candidate
tiling of the BFGS phase:
  * one group of G lanes per start, G a power of two from max(4, next_pow2(d))
    up to 64 (H in registers, 64/G starts per wavefront);
  * one 256-lane block per start (H in a device-memory slot).
Every tiling computes the same pairwise sums, so the tuner also checks that
all candidates return bit-identical results.  The fastest tiling of each probe
dimension covers the dimensions from the previous probe (exclusive) up to it;
runs of equal choices are merged into rules, written to csrc/zeus_tiling.inc
(rebuild the library afterwards).  The per-candidate times are kept in the
generated file's comments.
"""
import argparse
import datetime
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2603_28770_amd import workloads as W  # noqa: E402

OBJECTIVES = {"rosenbrock": 0, "rastrigin": 1, "ackley": 2, "styblinski_tang": 3}
PRECISIONS = {"fp64": 0, "mixed": 1}
DIMS = [2, 3, 4, 6, 8, 12, 16, 24, 32, 40, 48, 56, 64]
WIDE = 256


def candidates(d):
    g = 4
    while g < d:
        g *= 2
    out = []
    while g <= 64:
        out.append(g)
        g *= 2
    return out + [WIDE]


def probe_problem(obj, prec, d, quick):
    lo, hi = W.BOXES[obj]
    # about 2^22 coordinate-starts, at least 1024 starts
    n = max(1024, min(65536, (1 << (20 if quick else 22)) // (d * d)))
    return W.problem(objective=obj, dim=d, n=n, lower=lo, upper=hi, iter_pso=2, iter_bfgs=300,
                     seed=17, precision=prec, grad_tol=1e-4 if prec == "mixed" else 1e-6)


def time_tiling(Z, ctx, torch, p, lanes, reps):
    os.environ["ZEUS_TILE_LANES"] = str(lanes)
    try:
        ds = Z.DeviceSolve(p)
        stream = torch.cuda.Stream()
        ds.enqueue(ctx, stream.cuda_stream)  # warm-up
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ds.enqueue(ctx, stream.cuda_stream)
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts)), ds.host()
    finally:
        del os.environ["ZEUS_TILE_LANES"]


def rules_from(best):
    """best: {(obj, prec): [(d, lanes), ...] sorted by d} -> list of rules."""
    rules = []
    for (obj, prec), pts in sorted(best.items()):
        prev_d = 0
        cur = None
        for d, lanes in pts:
            lo = prev_d + 1
            if cur and cur[4] == lanes and cur[3] == lo - 1:
                cur[3] = d
            else:
                if cur:
                    rules.append(cur)
                cur = [OBJECTIVES[obj], PRECISIONS[prec], lo, d, lanes]
            prev_d = d
        if cur:
            rules.append(cur)
    # a rule may only name G >= every dimension it covers
    return [r for r in rules if r[4] == WIDE or r[4] >= r[3]]


def write_table(path, rules, notes):
    stamp = datetime.datetime.now(datetime.timezone.utc).strftime("%Y-%m-%d")
    lines = ["// zeus_tiling.inc -- tiling rules (see group_lanes).  Written by",
             f"// `python -m paper_2603_28770_amd.autotune` on {stamp}.",
             "// Columns: objective, precision, dmin, dmax, lanes per start (256: one block).",
             "// Median solve times (ms) per probe and candidate:"]
    lines += [f"//   {n}" for n in notes]
    lines += ["#pragma once", "static const zeus::TileRule kTileRules[] = {"]
    for r in rules:
        lines.append("    {%d, %d, %d, %d, %d}," % tuple(r))
    if not rules:
        lines.append("    {-1, -1, 0, -1, 0},  // placeholder: matches nothing")
    lines.append("};")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="fewer dimensions and smaller problems")
    ap.add_argument("--out", default=os.path.join(HERE, "csrc", "zeus_tiling.inc"))
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)
    import torch
    from paper_2603_28770_amd import zeus as Z
    ctx = Z.zeus_context_create(0)
    dims = [2, 4, 8, 16, 32, 48, 64] if args.quick else DIMS
    best, notes = {}, []
    t_start = time.time()
    for obj in OBJECTIVES:
        for prec in PRECISIONS:
            pts = []
            for d in dims:
                if obj == "rosenbrock" and d < 2:
                    continue
                p = probe_problem(obj, prec, d, args.quick)
                times, ref = {}, None
                for lanes in candidates(d):
                    t, out = time_tiling(Z, ctx, torch, p, lanes, args.reps)
                    times[lanes] = t
                    if ref is None:
                        ref = out
                    else:  # tiling-independent results
                        for k in ("f", "x", "iters", "status"):
                            if not np.array_equal(ref[k], out[k], equal_nan=True):
                                raise SystemExit(f"{obj} {prec} d={d}: tiling {lanes} changed {k}")
                choice = min(times, key=times.get)
                pts.append((d, choice))
                note = f"{obj} {prec} d={d} n={p['n']}: " + " ".join(
                    f"{k}:{v:.3f}" for k, v in times.items()) + f" -> {choice}"
                notes.append(note)
                print(note, flush=True)
            best[(obj, prec)] = pts
    rules = rules_from(best)
    write_table(args.out, rules, notes)
    Z.zeus_context_destroy(ctx)
    print(f"{len(rules)} rules -> {args.out} ({time.time() - t_start:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
