"""CPU runs under AddressSanitizer and UndefinedBehaviorSanitizer: both
builds of the oracle (gcc, with gcc's runtimes preloaded) under its pins, and
the library's host code (the C ABI's checks and planning, built by hipcc with
the sanitizers on the host pass only, clang's runtime preloaded) under the
ABI tests.  Each run is a child process, since a sanitizer runtime must be
loaded before the interpreter starts; a report or a failing test fails the
run."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

ORACLE_TESTS = ["tests/test_oracle_bfgs_pieces.py", "tests/test_oracle_lbfgs_window.py",
                "tests/test_oracle_pso.py", "tests/test_oracle_rng.py", "tests/test_oracle_hrow.py",
                "tests/test_oracle_required.py", "tests/test_oracle_readings.py"]


def _run(env_extra, tests):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", **env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", *tests], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


def test_oracle_under_asan_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True,
                           text=True).stdout.strip()
    if not (os.path.isabs(asan) and os.path.isabs(ubsan)):
        pytest.skip("gcc sanitizer runtimes not found")
    from oracle import build as OB
    OB.build_sanitized(str(tmp_path))
    out = _run({"LD_PRELOAD": f"{asan}:{ubsan}", "ZEUS_ORACLE_DIR": str(tmp_path)}, ORACLE_TESTS)
    assert " passed" in out


def test_host_api_under_asan_ubsan():
    rts = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rts:
        pytest.skip("clang's sanitizer runtime not found")
    from paper_2603_28770_amd import build as ZB
    if not os.path.exists(os.path.join(ZB.BUILD, "zeus_bfgs.o")):
        pytest.skip("the library's objects are not built")
    lib = ZB.build_sanitized()
    out = _run({"LD_PRELOAD": rts[0], "ZEUS_LIB": lib}, ["tests/test_abi_cpu.py"])
    assert " passed" in out
