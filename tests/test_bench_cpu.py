"""bench.py's host logic on the CPU: the single-GPU refusal, the algorithmic
flop counts against hand-computed cases, the mixed-precision split against
the whole count, and the reading of the committed rocprofv3 summaries (used
only while the kernel's sources still match them)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2603_28770_amd import rocprof_summary as RS  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_flops_hand_computed_rosenbrock_d2():
    # F_p = 8, F_s = 0, F_t = 13 at d = 2: gradient 8 + 2 * 13 = 34.
    # per start 34 + 4 = 38; per iteration 6 * 4 + 34 + 14 * 2 = 86;
    # per trial 8 + 4 = 12
    assert bench.algorithmic_flops("rosenbrock", 2, 1, 0, 0) == 38
    assert bench.algorithmic_flops("rosenbrock", 2, 1, 1, 0) == 38 + 86
    assert bench.algorithmic_flops("rosenbrock", 2, 1, 1, 1) == 38 + 86 + 12
    assert bench.algorithmic_flops("rosenbrock", 2, 3, 5, 7) == 3 * 38 + 5 * 86 + 7 * 12


def test_flops_hand_computed_lbfgs():
    # Rastrigin d = 4: F_p = 25, F_s = 4, F_t = 32, gradient 25 + 4 + 128 = 157;
    # two-loop direction with m = 3: 8 * 3 * 4 + 3 * 4 = 108
    per_iter = 108 + 157 + 14 * 4
    assert bench.algorithmic_flops("rastrigin", 4, 0, 1, 0, lbfgs_m=3) == per_iter


@pytest.mark.parametrize("obj,d", [("rosenbrock", 50), ("rastrigin", 10), ("ackley", 50),
                                   ("styblinski_tang", 128), ("sphere", 7), ("quartic", 3),
                                   ("goldstein_price", 2), ("poisson_fit", 4)])
def test_mixed_split_adds_up(obj, d):
    n, iters, trials = 1000, 12345, 67890
    for m in (0, 1, 8):
        w64, w32 = bench.algorithmic_flops_split(obj, d, n, iters, trials, m)
        assert w64 > 0 and w32 > 0
        assert w64 + w32 == bench.algorithmic_flops(obj, d, n, iters, trials, m)


def test_every_bench_workload_has_a_flop_model():
    for name, p in bench.WORKLOADS.items():
        assert bench.algorithmic_flops(p["objective"], p["dim"], p["n"], 10, 10) > 0, name
    for name, (p, model) in bench.USER_WORKLOADS.items():
        assert p["objective"] == "user"
        assert bench.algorithmic_flops(model, p["dim"], p["n"], 10, 10) > 0, name


@pytest.mark.parametrize("kernel,workload,stem", [
    ("bfgs_kernel", "rastrigin_d10_n65536", None),
    ("bfgs_kernel", "rosenbrock_d50_n131072", None),
    ("lbfgs_kernel", "rosenbrock_d200_n8192", "lbfgs_kernel_rosenbrock_d200_n8192_m8")])
def test_committed_profiles_parse(kernel, workload, stem):
    s = RS.load(os.path.join(ROOT, "profiles", f"{stem or kernel + '_' + workload}.md"))
    assert s is not None and s["workload"] == workload and s["kernel"] == kernel
    assert s["traffic_bytes"] == pytest.approx(s["read_bytes"] + s["write_bytes"])
    assert 0.0 < s["counter_fp64_tflops"] < 78.6
    assert 0.0 < s["valu_busy"] <= 1.0
    # bench uses the figures only while the kernel's sources still match
    current = s["sources_sha256"] == RS.sources_sha256(kernel)
    got = bench.profiled_traffic(workload, kernel, stem)
    assert got == (s["traffic_bytes"] if current else None)


def test_stale_profile_is_not_used(monkeypatch):
    monkeypatch.setattr(RS, "sources_sha256", lambda kernel: "0" * 64)
    assert bench.profile_figures("rastrigin_d10_n65536") is None
    assert bench.profiled_traffic("rastrigin_d10_n65536") is None


def test_missing_profile_is_not_used():
    assert bench.profiled_traffic("no_such_workload") is None


def test_method_count_hand_computed():
    # Rosenbrock d = 50: F_p = 392, F_t = 490; per iteration 6 * 2500 + 392 + 50 * 490;
    # per trial 392 + 100
    assert bench.method_flops("rosenbrock", 50, 1, 0) == 15000 + 392 + 24500
    assert bench.method_flops("rosenbrock", 50, 0, 1) == 492
    # Rastrigin d = 10: F_p = 60, F_t = 50
    assert bench.method_flops("rastrigin", 10, 3, 7) == 3 * (600 + 60 + 500) + 7 * (60 + 20)
    # Ackley d = 50: F_p = 353, F_t = 300
    assert bench.method_flops("ackley", 50, 1, 1) == 15000 + 353 + 15000 + 353 + 100
    # L-BFGS m = 8 at d = 200: the two-loop recursion in place of 6 d^2
    assert bench.method_flops("rosenbrock", 200, 1, 0, lbfgs_m=8) == (
        8 * 8 * 200 + 600 + 8 * 199 + 200 * 10 * 199)


def test_sparse_count_is_below_the_dense_one():
    assert bench.sparse_flops("rosenbrock", 50, 1, 0) == 15000 + 392 + 50 * 20
    for obj in ("rosenbrock", "rastrigin", "ackley", "styblinski_tang"):
        for d in (2, 10, 50, 200):
            assert bench.sparse_flops(obj, d, 100, 150) <= bench.method_flops(obj, d, 100, 150)
