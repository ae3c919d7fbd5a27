"""Benchmark: batched multistart (PSO -> BFGS) throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one whole solve of the workload (swarm initialisation, every PSO
update, the BFGS kernel over all starts, the best-of-N reduction) with its
state resident in HBM: the problem is handed over by value and the results
stay on the device.  Prints one JSON line.

value = BFGS start-iterations per second over the K timed steps (each
start-iteration is one gradient, one line search and one inverse-Hessian
update of one start).  Converged starts per second and the p50/p99 latency of
one solve are reported beside it.

roofline: the dominant kernel (the BFGS kernel) against the FP64 vector-ALU
peak of MI355X; its algorithmic flops per launch come from the method's
per-unit counts (``method_flops``: H work, one primal and d dense tangent
sweeps per iteration, one primal per line-search trial) and its launch
duration from HIP events on the stream it runs on.  ``algorithmic_flops``
recounts the same work from this code's own operation counts; the mixed-
precision line splits it into FP64 and FP32 work.

cpu_baseline: the CPU oracle (plain C, OpenMP over starts) timed on this
host on the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2603_28770_amd import workloads as W  # noqa: E402

METRIC = "converged starts/s & start-iters/s vs plain FP64; p50/p99 solve latency"
FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 157.3  # packed FP32 (two per lane per cycle)

WORKLOADS = {"rastrigin_d10_n65536": W.RASTRIGIN_D10, "rosenbrock_d2_n1024": W.ROSENBROCK_D2,
             "ackley_d50_n131072": W.ACKLEY_D50, "rosenbrock_d50_n131072": W.ROSENBROCK_D50,
             "styblinski_d128_n16384": W.STYBLINSKI_D128,
             "rosenbrock_d128_n16384": W.ROSENBROCK_D128,
             "rosenbrock_d200_n8192": W.ROSENBROCK_D200}


# Per-evaluation flop counts of the objectives as the kernels evaluate them
# (each +, -, x, / and each cos, sin, exp, sqrt counted as one flop):
#   primal(d)   flops of one value evaluation,
#   shared(d)   flops a dual evaluation adds once whatever the direction
#               (the sin of each cos term),
#   tangent(d)  flops one tangent direction adds.
def _counts(obj, d):
    if obj == "rosenbrock":
        return 8 * (d - 1), 0, 13 * (d - 1)
    if obj == "rastrigin":
        return 6 * d + 1, d, 8 * d
    if obj == "ackley":
        return 5 * d + 10, d, 7 * d + 9
    if obj == "styblinski_tang":
        return 7 * d + 1, 0, 11 * d + 1
    if obj == "sphere":
        return 2 * d + 1, 0, 4 * d + 1
    if obj == "quartic":
        return 3 * d, 0, 7 * d
    if obj == "goldstein_price":
        return 45, 0, 75
    if obj == "poisson_fit":  # per bin: 6 for the exponent, then exp, n e, -, +
        from paper_2603_28770_amd.user_objectives import POISSON_BINS
        return 10 * POISSON_BINS, 0, 10 * POISSON_BINS
    raise KeyError(obj)


def algorithmic_flops(obj, d, n_starts, total_iters, total_ls_trials, lbfgs_m=0):
    """Flops the method needs for a whole BFGS phase:
      per start:            one forward-mode gradient (primal + shared + d tangents)
                            and the norm test (2d);
      per start-iteration:  inverse-Hessian work 6 d^2 (one matrix-vector
                            product, rank-2 update with u = H g_new + p),
                            one gradient, vector work 14 d (g'p, y's, y'u,
                            ||g||^2, x + alpha p, s, y);
      per line-search trial: one primal evaluation and x + alpha p (2d).
    With L-BFGS (m pairs) the inverse-Hessian work is the two-loop recursion,
    2m dot products and 2m vector updates of 2d flops each plus the scaling
    (3d): 8 m d + 3d."""
    fp, fs, ft = _counts(obj, d)
    grad = fp + fs + d * ft
    h_work = 8 * lbfgs_m * d + 3 * d if lbfgs_m else 6 * d * d
    per_iter = h_work + grad + 14 * d
    return n_starts * (grad + 2 * d) + total_iters * per_iter + total_ls_trials * (fp + 2 * d)


def algorithmic_flops_split(obj, d, n_starts, total_iters, total_ls_trials, lbfgs_m=0):
    """The same work split by the precision the mixed mode computes it in:
    (FP64 flops: inverse-Hessian (or two-loop) and vector work, the trial
    points; FP32 flops: objective values and dual-number gradients)."""
    fp, fs, ft = _counts(obj, d)
    grad = fp + fs + d * ft
    h_work = 8 * lbfgs_m * d + 3 * d if lbfgs_m else 6 * d * d
    w32 = n_starts * grad + total_iters * grad + total_ls_trials * fp
    w64 = n_starts * 2 * d + total_iters * (h_work + 14 * d) + total_ls_trials * 2 * d
    return w64, w32


# Per-unit counts of the method's algorithmic work as this benchmark defines
# it for the roofline fraction: a primal evaluation F_p and the flops one
# dense tangent sweep adds, F_t, with each cos/exp/sqrt counted as one flop:
#   Rosenbrock       F_p = 8(d-1)        F_t = 10(d-1)
#   Rastrigin        F_p = 5d + d (cos)  F_t = 5d
#   Ackley           F_p = 6d + d (cos) + 2 (exp) + 1 (sqrt)   F_t = 6d
#   Styblinski-Tang  F_p = 7d            F_t = 6d
# (the test-only and user objectives take this file's own counts above).
def _method_counts(obj, d):
    if obj == "rosenbrock":
        return 8 * (d - 1), 10 * (d - 1)
    if obj == "rastrigin":
        return 6 * d, 5 * d
    if obj == "ackley":
        return 7 * d + 3, 6 * d
    if obj == "styblinski_tang":
        return 7 * d, 6 * d
    fp, fs, ft = _counts(obj, d)
    return fp + fs, ft


# Tangent flops per direction when only the terms that hold x_j are swept
# (each direction of Alg. 5 has at most two nonzero term tangents for
# Rosenbrock, one for the separable objectives; Ackley adds the outer chain
# of its two sums).
_SPARSE_TANGENT = {"rosenbrock": 20, "rastrigin": 5, "ackley": 14, "styblinski_tang": 6,
                   "sphere": 2, "quartic": 3}


def method_flops(obj, d, total_iters, total_ls_trials, lbfgs_m=0):
    """The method's algorithmic work, per start-iteration W_H + W_grad + W_LS:
    W_H = 6 d^2 (one matrix-vector product and the rank-2 update; with L-BFGS
    the two-loop recursion 8 m d + 3 d), W_grad = F_p + d F_t (one primal and
    the d dense tangent sweeps of Alg. 5), and per line-search trial
    F_p + 2 d."""
    fp, ft = _method_counts(obj, d)
    h_work = 8 * lbfgs_m * d + 3 * d if lbfgs_m else 6 * d * d
    return total_iters * (h_work + fp + d * ft) + total_ls_trials * (fp + 2 * d)


def sparse_flops(obj, d, total_iters, total_ls_trials, lbfgs_m=0):
    """The same work with each gradient direction sweeping only the terms
    that hold its coordinate (what a term-parallel evaluation needs); for
    objectives without a term structure the dense count."""
    fp, ft = _method_counts(obj, d)
    tan = _SPARSE_TANGENT.get(obj)
    grad = fp + d * (min(tan, ft) if tan is not None else ft)
    h_work = 8 * lbfgs_m * d + 3 * d if lbfgs_m else 6 * d * d
    return total_iters * (h_work + grad) + total_ls_trials * (fp + 2 * d)


def main_kernel(p):
    """The kernel that runs the BFGS phase of problem p, and the name its
    rocprofv3 summary carries under profiles/ (kernel_workload[_mM].md)."""
    if p.get("lbfgs_m", 0):
        return "lbfgs_kernel", f"lbfgs_kernel_{p['name']}_m{p['lbfgs_m']}"
    if p["dim"] <= 64:
        kernel = "bfgs_kernel"
    else:  # one block per start: H in registers up to d = 128, in registers and LDS
        # up to 208, in device memory above
        kernel = ("bfgs_tile_kernel" if p["dim"] <= 128 else
                  "bfgs_hybrid_kernel" if p["dim"] <= 208 else "bfgs_wide_kernel")
    return kernel, f"{kernel}_{p['name']}"


def profile_figures(workload, kernel="bfgs_kernel", stem=None):
    """The JSON block of the committed rocprofv3 summary of `kernel` on this
    workload (profiles/<stem>.md, stem = kernel_workload by default), or None
    when there is none or the kernel's sources have changed since it was
    taken."""
    from paper_2603_28770_amd import rocprof_summary as RS
    s = RS.load(os.path.join(ROOT, "profiles", f"{stem or kernel + '_' + workload}.md"))
    if not s or kernel not in RS.KERNEL_SOURCES or s.get("sources_sha256") != RS.sources_sha256(kernel):
        return None
    return s


def profiled_traffic(workload, kernel="bfgs_kernel", stem=None):
    """HBM bytes per launch of `kernel` on this workload (FETCH_SIZE +
    WRITE_SIZE scaled by a copy kernel's), from the committed summary while it
    is current, else None."""
    s = profile_figures(workload, kernel, stem)
    return s.get("traffic_bytes") if s else None


def cpu_baseline(p, sub=256, sub1=None):
    """The oracle on the full workload: its sequential PSO, then BFGS from every
    start with OpenMP over starts on all threads it is given (above d = 20
    from `sub` strided starts; on one thread from `sub1`, default 1024 up to
    d = 20 and 64 above)."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    sw = O.pso(p)
    t1 = time.perf_counter()
    idx = None
    if p["dim"] > 20:  # large problems: a strided subset of starts (exact per start)
        idx = W.strided_subset(p["n"], sub)
    r = O.bfgs(p, sw["x"], idx=idx)
    t2 = time.perf_counter()
    m = p["n"] if idx is None else idx.size
    per_start = (t1 - t0) / p["n"] + (t2 - t1) / m
    iters_per_start = float(r["iters"].mean())
    sample = (f"full swarm ({p['n']} particles, {p['iter_pso']} updates, sequential) then BFGS "
              f"from {m} of {p['n']} starts; {t1 - t0:.2f} s swarm + {t2 - t1:.2f} s BFGS")
    # one core: the same swarm (sequential already) and BFGS on one thread
    # over a strided subset of the starts
    idx1 = W.strided_subset(p["n"], sub1 or (1024 if p["dim"] <= 20 else 64))
    t3 = time.perf_counter()
    r1 = O.bfgs(p, sw["x"], idx=idx1, nthreads=1)
    t4 = time.perf_counter()
    per_start1 = (t1 - t0) / p["n"] + (t4 - t3) / idx1.size
    return {"value": iters_per_start / per_start, "unit": "start-iters/s",
            "cores": int(r["threads"]), "kind": "oracle", "sample": sample,
            "converged_starts_per_s": float(np.mean(r["status"] == 1)) / per_start,
            "value_1core": float(r1["iters"].mean()) / per_start1,
            "sample_1core": f"the same swarm, then BFGS on one thread from {idx1.size} strided starts; "
                            f"{t4 - t3:.2f} s"}


MULTI = ("uneven_batch", "served_mix")
HEADLINE = "rosenbrock_d50_n131072"
SECONDARY = ("ackley_d50_n131072", "rastrigin_d10_n65536")


def _user_source(name):
    from paper_2603_28770_amd import user_objectives as UO
    return UO.poisson_fit_source() if name == "poisson_fit" else getattr(UO, name.upper())


# user-code workloads: problem, the objective its source restates (for the
# flop counts), the source
USER_WORKLOADS = {"user_rosenbrock_d50_n131072": (W.USER_ROSENBROCK_D50, "rosenbrock"),
                  "user_rosenbrock_d50_n131072_mixed": (W.USER_ROSENBROCK_D50_MIXED, "rosenbrock"),
                  "user_rosenbrock_d200_n8192_lbfgs8": (W.USER_ROSENBROCK_D200_LBFGS, "rosenbrock"),
                  "user_poisson_fit_n65536": (W.USER_POISSON_FIT, "poisson_fit")}


def _totals(outs, reqs):
    iters = sum(o["summary"]["total_iters"] for o in outs)
    conv = sum(o["summary"]["n_converged"] for o in outs)
    starts = sum(int(p["n"]) for p in reqs)
    succ = sum(int(np.sum(o["f"] - W.f_star(p["objective"], p["dim"]) < 1e-4))
               for o, p in zip(outs, reqs))
    return iters, conv, starts, succ / max(1, starts)


def _mix_config(name, reqs, scale):
    dims = [int(p["dim"]) for p in reqs]
    return {"workload": name, "requests": len(reqs), "starts": sum(int(p["n"]) for p in reqs),
            "dim_range": [min(dims), max(dims)], "n_scale": scale,
            "iter_bfgs": int(reqs[0]["iter_bfgs"])}


def run_uneven_batch(args, Z, ctx):
    """The uneven batch (512 requests, d in [2,128], N log-uniform in
    [256, 16384]) through one zeus_minimize_batch call, FP64 and mixed.  The
    timed region includes copying every result to host memory."""
    scale = args.n_scale if args.n_scale else 1.0
    reqs = [W.scaled(p, max(1, int(p["n"] * scale))) for p in W.uneven_batch()]
    # warm-up: the same batch, so that the first launches load the code
    # objects and the context sizes its device buffers outside the timed call
    Z.zeus_minimize_batch(ctx, reqs)
    t0 = time.perf_counter()
    outs = Z.zeus_minimize_batch(ctx, reqs)
    t = time.perf_counter() - t0
    print(f"[batch] fp64: {t:.2f} s", file=sys.stderr, flush=True)
    iters, conv, starts, succ = _totals(outs, reqs)
    mreqs = [dict(p, precision="mixed", grad_tol=1e-4) for p in reqs]
    t0 = time.perf_counter()
    mouts = Z.zeus_minimize_batch(ctx, mreqs)
    tm = time.perf_counter() - t0
    miters, mconv, _, msucc = _totals(mouts, mreqs)
    return {
        "metric": METRIC, "value": iters / t, "unit": "start-iters/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": t * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded Philox request stream)",
        "config": _mix_config("uneven_batch", reqs, scale),
        "converged_starts_per_s": conv / t, "start_iters": iters, "success_rate": succ,
        "mixed": {"grad_tol": 1e-4, "ms": tm * 1e3, "start_iters_per_s": miters / tm,
                  "converged_starts_per_s": mconv / tm, "success_rate": msucc,
                  "speedup_vs_fp64": t / tm},
        "roofline": None, "note": "multi-request workload; the roofline is reported on the "
                                  "single-problem default workload"}


def run_served_mix(args, Z, ctx, compact=False):
    """The served mix (d in [2,200], N log-uniform; mixed precision, Theta 1e-4)
    at reduced size: plain FP64 one request at a time, then the server closed
    loop (all submitted at once: saturation rate mu), then Poisson arrivals at
    0.5, 0.7 and 0.9 mu with per-request latency t_done - t_submit.  With
    compact=True returns the comparison block the default line nests."""
    import torch
    count = args.requests or 256
    scale = args.n_scale if args.n_scale else 1.0 / 16
    base = W.served_mix(count)
    reqs = [W.scaled(p, max(1, int(p["n"] * scale))) for p in base]
    fp64 = [dict(p, precision="fp64") for p in reqs]
    Z.zeus_minimize(ctx, fp64[0])  # warm-up
    t0 = time.perf_counter()
    souts = [Z.zeus_minimize(ctx, p) for p in fp64]
    t_seq = time.perf_counter() - t0
    print(f"[served] fp64 one at a time: {t_seq:.2f} s", file=sys.stderr, flush=True)
    s_iters, s_conv, starts, s_succ = _totals(souts, fp64)
    free, _ = torch.cuda.mem_get_info()
    budget = max(1 << 30, free - (8 << 30))
    with Z.Server(ctx, budget) as srv:
        t0 = time.perf_counter()
        ts = [srv.submit(p) for p in reqs]
        outs = [srv.wait(t) for t in ts]
        t_closed = time.perf_counter() - t0
        iters, conv, _, succ = _totals(outs, reqs)
        mu = count / t_closed
        print(f"[served] closed loop: {t_closed:.2f} s ({mu:.1f} req/s)", file=sys.stderr, flush=True)
        rng = np.random.Generator(np.random.Philox(key=[4, int.from_bytes(b"ARR", "little")]))
        open_loop = {}
        for frac in (0.5, 0.7, 0.9):
            lam = frac * mu
            arrive = np.cumsum(rng.exponential(1.0 / lam, count))
            tickets = [None] * count

            def feeder():
                start = time.perf_counter()
                for k in range(count):
                    delay = start + arrive[k] - time.perf_counter()
                    if delay > 0:
                        time.sleep(delay)
                    tickets[k] = srv.submit(reqs[k])

            import threading
            th = threading.Thread(target=feeder)
            t0 = time.perf_counter()
            th.start()
            res = []
            for k in range(count):
                while tickets[k] is None:
                    time.sleep(1e-4)
                res.append(srv.wait(tickets[k]))
            th.join()
            span = time.perf_counter() - t0
            print(f"[served] open loop at {frac} mu: {span:.2f} s", file=sys.stderr, flush=True)
            lat = np.array([(o["times"]["t_done_ns"] - o["times"]["t_submit_ns"]) / 1e6 for o in res])
            oi, oc, _, osc = _totals(res, reqs)
            open_loop[f"{frac:.1f}"] = {
                "rate_req_per_s": lam, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "start_iters_per_s": oi / span,
                "converged_starts_per_s": oc / span, "success_rate": osc}
    main_ol = open_loop["0.7"]
    if compact:
        return {"config": _mix_config("served_mix", reqs, scale), "precision": "mixed",
                "grad_tol": float(reqs[0]["grad_tol"]),
                "fp64_one_at_a_time_ms": t_seq * 1e3, "served_closed_loop_ms": t_closed * 1e3,
                "speedup_vs_fp64_one_at_a_time": t_seq / t_closed,
                "success_rate": succ, "fp64_success_rate": s_succ,
                "equal_success": bool(abs(succ - s_succ) <= 0.01),
                "start_iters_per_s": iters / t_closed, "converged_starts_per_s": conv / t_closed,
                "fp64_start_iters_per_s": s_iters / t_seq,
                "saturation_req_per_s": mu, "p50_solve_ms": main_ol["p50_ms"],
                "p99_solve_ms": main_ol["p99_ms"], "open_loop": open_loop}
    return {
        "metric": METRIC, "value": iters / t_closed, "unit": "start-iters/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": t_closed * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64 (mixed)",
        "data": "synthetic (seeded Philox request stream, Poisson arrivals)",
        "config": _mix_config("served_mix", reqs, scale),
        "converged_starts_per_s": conv / t_closed, "success_rate": succ,
        "saturation_req_per_s": mu, "p50_solve_ms": main_ol["p50_ms"],
        "p99_solve_ms": main_ol["p99_ms"], "open_loop": open_loop,
        "fp64_one_at_a_time": {"ms": t_seq * 1e3, "start_iters_per_s": s_iters / t_seq,
                               "converged_starts_per_s": s_conv / t_seq, "success_rate": s_succ},
        "speedup_vs_fp64_one_at_a_time": t_seq / t_closed,
        "roofline": None, "note": "multi-request workload; the roofline is reported on the "
                                  "single-problem default workload"}


def run_user(args, Z, ctx):
    """A user objective: compiled once (zeus_objective_compile, timed apart),
    then K solves through the blocking zeus_minimize_user, whose results are
    copied to host memory inside the timed region.  Kernel times come from
    HIP events on the context's stream; the roofline uses the BFGS kernel's.
    A user restatement of a built-in objective is timed beside the built-in
    one on the same problem, which prices the whole-form evaluation."""
    p, model = USER_WORKLOADS[args.workload]
    t0 = time.perf_counter()
    obj = Z.zeus_objective_compile(ctx, _user_source(model))
    t_compile = time.perf_counter() - t0

    def timed(solve):
        for _ in range(args.warmup):
            solve()
        Z.zeus_context_set_profiling(ctx, True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = solve()
        wall = time.perf_counter() - t0
        prof = Z.zeus_context_get_profile(ctx)
        Z.zeus_context_set_profiling(ctx, False)
        return wall * 1e3 / args.steps, prof, out

    ms, prof, out = timed(lambda: Z.zeus_minimize_user(ctx, obj, [p])[0])
    Z.zeus_objective_destroy(obj)
    s = out["summary"]
    iters = s["total_iters"]
    bfgs_ms = prof["bfgs_ms"] / max(1, prof["bfgs_launches"])
    lm = p.get("lbfgs_m", 0)
    flops = method_flops(model, p["dim"], iters, s["total_ls_trials"], lm)
    achieved = flops / (bfgs_ms * 1e-3) / 1e12
    line = {
        "metric": METRIC, "value": iters / (ms / 1e3), "unit": "start-iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded Philox starts in the box; user objective compiled at run time)",
        "config": {"workload": args.workload, "objective": f"user ({model})", "dim": p["dim"],
                   "n_starts": p["n"], "iter_pso": p["iter_pso"], "iter_bfgs": p["iter_bfgs"],
                   "grad_tol": p["grad_tol"], "precision": "fp64",
                   "method": f"lbfgs_m{lm}" if lm else "bfgs"},
        "compile_s": t_compile,
        "converged_starts_per_s": s["n_converged"] / (ms / 1e3),
        "start_iters_per_step": iters, "ls_trials_per_iter": s["total_ls_trials"] / max(1, iters),
        "n_converged": s["n_converged"], "best_f": s["best_f"],
        "kernel_ms": {"pso": prof["pso_ms"] / args.steps, "bfgs": bfgs_ms,
                      "reduce": prof["reduce_ms"] / args.steps},
        # swarm particle-iterations (initialisation + iter_pso sweeps) per
        # second of the swarm kernels
        "pso_particle_iters_per_s": p["n"] * (p["iter_pso"] + 1)
                                    / max(1e-9, prof["pso_ms"] / args.steps * 1e-3),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VALU_PEAK_TFLOPS,
                     "traffic": None,
                     "kernel": f"{'lbfgs' if lm else 'bfgs'}_kernel (user objective)",
                     "flops_per_launch": flops},
        "note": "blocking entry point: ms_per_step includes copying the results to host memory",
    }
    if p.get("precision") == "mixed":
        # t_ideal = W64 / FP64 peak + W32 / FP32 peak; the peak is this mix's
        # blend of the two, so that frac = achieved / peak = t_ideal / t
        w64, w32 = algorithmic_flops_split(model, p["dim"], p["n"], iters, s["total_ls_trials"], lm)
        t_ideal = w64 / (FP64_VALU_PEAK_TFLOPS * 1e12) + w32 / (FP32_VALU_PEAK_TFLOPS * 1e12)
        blend = (w64 + w32) / t_ideal / 1e12
        line["dtype"] = "f32+f64 (mixed)"
        line["config"]["precision"] = "mixed"
        line["roofline"].update(achieved=(w64 + w32) / (bfgs_ms * 1e-3) / 1e12, peak=blend,
                                frac=t_ideal * 1e3 / bfgs_ms, w64_flops=w64, w32_flops=w32,
                                flops_per_launch=w64 + w32)
        line["note"] += "; the CPU baseline is the oracle, which computes in FP64"
    if model in W.BOXES:  # a restated built-in objective: the built-in beside it
        pb = dict(p, objective=model)
        bms, bprof, bout = timed(lambda: Z.zeus_minimize(ctx, pb))
        b_bfgs = bprof["bfgs_ms"] / max(1, bprof["bfgs_launches"])
        line["builtin"] = {"objective": model, "ms_per_step": bms, "bfgs_ms": b_bfgs,
                           "start_iters_per_step": bout["summary"]["total_iters"],
                           "n_converged": bout["summary"]["n_converged"],
                           "user_over_builtin_bfgs_time": bfgs_ms / b_bfgs}
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        from oracle import user as OU
        OU.use(_user_source(model), O.lib())   # the same source, built for the CPU
        # whole-form gradients cost d evaluations: fewer sampled starts above d = 64
        line["cpu_baseline"] = cpu_baseline(p, 64, 8) if p["dim"] > 64 else cpu_baseline(p)
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=None,
                    choices=sorted(WORKLOADS) + list(MULTI) + sorted(USER_WORKLOADS),
                    help="one workload only (default: the d = 50 Rosenbrock headline with "
                         "Ackley d = 50, Rastrigin d = 10 and the served set beside it)")
    ap.add_argument("--n-scale", type=float, default=0.0,
                    help="multi-request workloads: multiply every request's start count")
    ap.add_argument("--requests", type=int, default=0, help="served_mix: number of requests")
    ap.add_argument("--lbfgs-m", type=int, default=0, metavar="M",
                    help="solve the workload with L-BFGS keeping M pairs (default: BFGS)")
    ap.add_argument("--required-c", type=int, default=0, metavar="C",
                    help="also time the solve with early stop at C converged starts (the "
                         "paper's time-to-C-convergences metric; asynchronous entry point)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-served", action="store_true",
                    help="default run: skip the served mixed-precision set")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision run of the same workload")
    ap.add_argument("--study", choices=("ncorrect_vs_d", "pso_iters"), default=None,
                    help="effectiveness study instead of the throughput line: N_correct per "
                         "Rastrigin dimension (10^5 particles, 5 sweeps, stop at 100 "
                         "convergences), or N_correct and time to 100 convergences per number "
                         "of swarm sweeps (d = 5 Rastrigin and Rosenbrock)")
    ap.add_argument("--runs", type=int, default=100, help="--study: runs per configuration")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 3 times (a plain copy kernel "
                         "of known size for scaling FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 8, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); "
              "multi-GPU sharding is a design note, not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_28770_amd import zeus as Z

    if args.study:
        from paper_2603_28770_amd import studies as S
        ctx = Z.zeus_context_create(0)
        log = lambda s: print(s, file=sys.stderr, flush=True)  # noqa: E731
        if args.study == "ncorrect_vs_d":
            rows = S.sweep(Z, ctx, "rastrigin", [(d, 5) for d in range(1, 11)], args.runs,
                           100000, 100, 1000, log)
        else:
            sweeps = [0, 1, 2, 5, 10, 20, 50]
            rows = []
            for obj in ("rastrigin", "rosenbrock"):
                rows += S.sweep(Z, ctx, obj, [(5, k) for k in sweeps], args.runs, 100000, 100,
                                2000, log)
        Z.zeus_context_destroy(ctx)
        print(json.dumps({"study": args.study, "data": "synthetic (seeded Philox starts)",
                          "criterion": "Euclidean distance to the global minimiser < 0.5",
                          "rows": rows}), flush=True)
        return

    if args.workload in MULTI or args.workload in USER_WORKLOADS:
        ctx = Z.zeus_context_create(0)
        run = {"uneven_batch": run_uneven_batch, "served_mix": run_served_mix}.get(
            args.workload, run_user)
        line = run(args, Z, ctx)
        Z.zeus_context_destroy(ctx)
        print(json.dumps(line), flush=True)
        return

    ctx = Z.zeus_context_create(0)
    stream = torch.cuda.Stream()   # the library's kernels and torch's events share it
    if args.workload:
        p = WORKLOADS[args.workload]
        if args.lbfgs_m:
            p = dict(p, lbfgs_m=args.lbfgs_m)
        line = measure_single(args, Z, ctx, stream, p, args.workload)
        if args.required_c > 0:
            line["time_to_c"] = time_to_c(Z, ctx, stream, p, args.required_c, max(1, args.steps),
                                          max(1, args.warmup))
        Z.zeus_context_destroy(ctx)
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = cpu_baseline(p)
        print(json.dumps(line), flush=True)
        return

    # default: the d = 50 Rosenbrock problem (the largest single problem) in
    # FP64 as the headline, with Ackley d = 50, the d = 10 Rastrigin problem
    # and the served mixed-precision set against plain FP64 beside it
    head = HEADLINE
    line = measure_single(args, Z, ctx, stream, WORKLOADS[head], head)
    also = {}
    for name in SECONDARY:
        r = measure_single(args, Z, ctx, stream, WORKLOADS[name], name)
        also[name] = {k: r[k] for k in ("value", "unit", "ms_per_step", "converged_starts_per_s",
                                        "p50_solve_ms", "p99_solve_ms", "success_rate",
                                        "best_f", "ls_trials_per_iter", "kernel_ms", "roofline",
                                        "mixed", "config") if k in r}
        print(f"[bench] {name}: {r['value']:.4g} start-iters/s", file=sys.stderr, flush=True)
    line["also"] = also
    if not args.no_served:
        line["served"] = run_served_mix(args, Z, ctx, compact=True)
    Z.zeus_context_destroy(ctx)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(WORKLOADS[head])
    print(json.dumps(line), flush=True)


def measure_single(args, Z, ctx, stream, p, name):
    """One problem on the device: K eager solves through the async entry
    point (state resident in HBM) timed with HIP events on `stream`, the same
    solve replayed from a captured HIP graph, and (FP64 problems) the mixed-
    precision solve.  Returns the JSON line of the problem."""
    import torch
    sptr = stream.cuda_stream

    def timed(problem):
        ds = Z.DeviceSolve(problem)
        for _ in range(args.warmup):
            ds.enqueue(ctx, sptr)
        torch.cuda.synchronize()
        Z.zeus_context_set_profiling(ctx, True)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b in evs:
            a.record(stream)
            ds.enqueue(ctx, sptr)
            b.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = Z.zeus_context_get_profile(ctx)
        Z.zeus_context_set_profiling(ctx, False)
        lat = np.array([a.elapsed_time(b) for a, b in evs])
        return wall, prof, lat, ds.host()

    wall, prof, lat, out = timed(p)
    s = out["summary"]

    # the same solve captured once into a HIP graph and replayed
    plan = Z.DevicePlan(ctx, [p])
    for _ in range(args.warmup):
        plan.launch(sptr)
    torch.cuda.synchronize()
    gevs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in gevs:
        a.record(stream)
        plan.launch(sptr)
        b.record(stream)
    torch.cuda.synchronize()
    gwall = time.perf_counter() - t0
    glat = np.array([a.elapsed_time(b) for a, b in gevs])
    gout = plan.host()[0]
    plan.close()
    graph = {"ms_per_step": gwall * 1e3 / args.steps,
             "p50_solve_ms": float(np.percentile(glat, 50)),
             "p99_solve_ms": float(np.percentile(glat, 99)),
             "same_results": bool(np.array_equal(gout["f"], out["f"], equal_nan=True)
                                  and gout["summary"] == s)}
    ms_per_step = wall * 1e3 / args.steps
    fstar = W.f_star(p["objective"], p["dim"])
    success = float(np.mean(out["f"] - fstar < 1e-4))
    mixed = None
    if not args.no_mixed and p.get("precision", "fp64") == "fp64":
        pm = dict(p, precision="mixed", grad_tol=max(p["grad_tol"], 1e-4))
        mwall, mprof, mlat, mout = timed(pm)
        ms = mout["summary"]
        mms = mwall * 1e3 / args.steps
        msucc = float(np.mean(mout["f"] - fstar < 1e-4))
        mixed = {"grad_tol": pm["grad_tol"], "ms_per_step": mms,
                 "start_iters_per_s": ms["total_iters"] / (mms / 1e3),
                 "converged_starts_per_s": ms["n_converged"] / (mms / 1e3),
                 "p50_solve_ms": float(np.percentile(mlat, 50)),
                 "p99_solve_ms": float(np.percentile(mlat, 99)),
                 "success_rate": msucc, "fp64_success_rate": success,
                 "speedup_vs_fp64": ms_per_step / mms,
                 "equal_success": bool(abs(msucc - success) <= 0.01)}
        # t_ideal = W64 / FP64 peak + W32 / FP32 peak, against the BFGS kernel's time
        m_bfgs = mprof["bfgs_ms"] / max(1, mprof["bfgs_launches"])
        w64, w32 = algorithmic_flops_split(pm["objective"], pm["dim"], pm["n"], ms["total_iters"],
                                           ms["total_ls_trials"], pm.get("lbfgs_m", 0))
        t_ideal = w64 / (FP64_VALU_PEAK_TFLOPS * 1e12) + w32 / (FP32_VALU_PEAK_TFLOPS * 1e12)
        mixed["roofline"] = {"bound": "alu", "bfgs_ms": m_bfgs, "w64_flops": w64, "w32_flops": w32,
                             "peak_fp64": FP64_VALU_PEAK_TFLOPS, "peak_fp32": FP32_VALU_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "t_ideal_ms": t_ideal * 1e3,
                             "frac": t_ideal * 1e3 / m_bfgs}

    iters = s["total_iters"]
    value = iters / (ms_per_step / 1e3)
    conv_per_s = s["n_converged"] / (ms_per_step / 1e3)
    bfgs_ms = prof["bfgs_ms"] / max(1, prof["bfgs_launches"])
    lm = p.get("lbfgs_m", 0)
    trials = s["total_ls_trials"]
    flops = method_flops(p["objective"], p["dim"], iters, trials, lm)
    sparse = sparse_flops(p["objective"], p["dim"], iters, trials, lm)
    kernel, stem = main_kernel(p)
    achieved = flops / (bfgs_ms * 1e-3) / 1e12
    line = {
        "metric": METRIC, "value": value, "unit": "start-iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded Philox starts in the box; analytic objective)",
        "config": {"workload": name, "objective": p["objective"], "dim": p["dim"],
                   "n_starts": p["n"], "iter_pso": p["iter_pso"], "iter_bfgs": p["iter_bfgs"],
                   "grad_tol": p["grad_tol"], "precision": p.get("precision", "fp64"),
                   "method": f"lbfgs_m{lm}" if lm else "bfgs"},
        "converged_starts_per_s": conv_per_s,
        "p50_solve_ms": float(np.percentile(lat, 50)), "p99_solve_ms": float(np.percentile(lat, 99)),
        "start_iters_per_step": iters, "ls_trials_per_iter": trials / max(1, iters),
        "n_converged": s["n_converged"], "best_f": s["best_f"], "success_rate": success,
        "kernel_ms": {"pso": prof["pso_ms"] / args.steps, "bfgs": bfgs_ms,
                      "reduce": prof["reduce_ms"] / args.steps},
        # swarm particle-iterations (initialisation + iter_pso sweeps) per
        # second of the swarm kernels
        "pso_particle_iters_per_s": p["n"] * (p["iter_pso"] + 1)
                                    / max(1e-9, prof["pso_ms"] / args.steps * 1e-3),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VALU_PEAK_TFLOPS,
                     "traffic": profiled_traffic(name, kernel, stem), "kernel": kernel,
                     "flops_per_launch": flops, "count": "method (dense tangent sweeps)",
                     "sparse_achieved": sparse / (bfgs_ms * 1e-3) / 1e12,
                     "sparse_frac": sparse / (bfgs_ms * 1e-3) / 1e12 / FP64_VALU_PEAK_TFLOPS},
    }
    pf = profile_figures(name, kernel, stem)
    if pf and "counter_fp64_tflops" in pf:
        # FP64 work the SQ counters saw (every lane of a wave, padding included)
        line["roofline"]["counter_achieved"] = pf["counter_fp64_tflops"]
        line["roofline"]["counter_frac"] = pf["counter_fp64_tflops"] / FP64_VALU_PEAK_TFLOPS
        line["roofline"]["valu_busy"] = pf.get("valu_busy")
    line["graph"] = graph
    if mixed is not None:
        line["mixed"] = mixed
    return line


def time_to_c(Z, ctx, stream, p, required_c, reps, warmup):
    """Time to required_c convergences (the paper's time metric) against the
    full solve: both enqueued through the asynchronous entry point with state
    resident in HBM, timed with HIP events on `stream`; the stop is decided
    on the device."""
    import torch
    sptr = stream.cuda_stream

    def timed(problem):
        ds = Z.DeviceSolve(problem)
        for _ in range(warmup):
            ds.enqueue(ctx, sptr)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(reps)]
        for a, b in evs:
            a.record(stream)
            ds.enqueue(ctx, sptr)
            b.record(stream)
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in evs])), ds.host()

    t_full, full = timed(p)
    t_early, early = timed(dict(p, required_converged=required_c))
    return {"required_c": required_c, "ms": t_early, "full_solve_ms": t_full,
            "speedup": t_full / t_early, "k_star": int(early["iters"].max()),
            "converged": int(np.sum(early["status"] == 1)),
            "stopped": int(np.sum(early["status"] == 2)),
            "full_converged": int(np.sum(full["status"] == 1)),
            "start_iters": int(early["summary"]["total_iters"]),
            "full_start_iters": int(full["summary"]["total_iters"])}


if __name__ == "__main__":
    main()
