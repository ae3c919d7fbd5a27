"""CPU-only checks of the C ABI library: it loads, exports every entry point
declared in include/zeus.h, its struct layouts match the header as compiled
by gcc, and argument validation behaves as documented (no GPU needed)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zeus.h")


@pytest.fixture(scope="module")
def Z():
    from paper_2603_28770_amd import zeus
    return zeus


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(zeus_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(Z):
    names = _declared()
    assert len(names) >= 11
    out = subprocess.run(["nm", "-D", "--defined-only", Z.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (zeus_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert set(Z.EXPORTS) == set(names)


def test_trace_ranges_are_linked(Z):
    """The entry points and launch phases mark roctx ranges (rocprofv3
    --marker-trace): the library takes the roctx calls from ROCm's roctx
    library, and the range names are in its code."""
    und = subprocess.run(["nm", "-D", "--undefined-only", Z.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    for sym in ("roctxRangePushA", "roctxRangePop", "roctxMarkA"):
        assert sym in und, sym
    data = open(Z.LIB_PATH, "rb").read()
    for name in (b"zeus_minimize_batch", b"zeus.swarm", b"zeus.bfgs", b"zeus.server.step",
                 b"zeus.server.admit", b"zeus.server.retire", b"zeus_plan_launch"):
        assert name + b"\0" in data, name


def test_struct_layouts_match_header(Z, tmp_path):
    import ctypes as C
    prog = tmp_path / "layout.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "zeus.h"\n'
                    "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu\\n\","
                    "sizeof(zeus_problem), sizeof(zeus_result), sizeof(zeus_summary),"
                    "sizeof(zeus_profile), offsetof(zeus_problem, seed),"
                    "offsetof(zeus_result, summary), offsetof(zeus_problem, grad_tol),"
                    "offsetof(zeus_result, resets));return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog), "-o",
                    str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals == [C.sizeof(Z.zeus_problem), C.sizeof(Z.zeus_result),
                    C.sizeof(Z.zeus_summary), C.sizeof(Z.zeus_profile),
                    Z.zeus_problem.seed.offset, Z.zeus_result.summary.offset,
                    Z.zeus_problem.grad_tol.offset, Z.zeus_result.resets.offset]


def test_version(Z):
    assert Z.zeus_abi_version() == Z.ABI_VERSION == 2 and "gfx950" in Z.zeus_version()


def _p(**kw):
    from paper_2603_28770_amd import workloads as W
    p = W.problem(objective="rastrigin", dim=10, n=1000, lower=-5.12, upper=5.12, iter_pso=3)
    p.update(kw)
    return p


@pytest.mark.parametrize("bad", [dict(dim=0), dict(n=0), dict(lower=1.0, upper=1.0),
                                 dict(upper=float("nan")), dict(iter_ls=0),
                                 dict(iter_bfgs=-1), dict(iter_pso=-1), dict(grad_tol=0.0),
                                 dict(grad_tol=float("inf")), dict(armijo_c=0.0),
                                 dict(armijo_c=1.0), dict(ls_shrink=1.0), dict(c1=float("inf")),
                                 dict(objective="rosenbrock", dim=1),
                                 dict(objective="goldstein_price", dim=3),
                                 dict(required_converged=-1)])
def test_validation_rejects(Z, bad):
    assert Z.zeus_validate(Z.make_problem(_p())) == Z.OK
    pb = Z.make_problem(_p(**bad))
    assert Z.zeus_validate(pb) == Z.EINVAL
    assert Z.zeus_last_error() != ""


def test_validation_abi_and_history(Z):
    pb = Z.make_problem(_p())
    pb.abi_version = 1  # the layout before the per-start skip and reset counts
    assert Z.zeus_validate(pb) == Z.EINVAL
    for m, code in ((-1, Z.EINVAL), (0, Z.OK), (1, Z.OK), (8, Z.OK), (9, Z.EUNSUPPORTED)):
        pb = Z.make_problem(_p())
        pb.lbfgs_m = m
        assert Z.zeus_validate(pb) == code, m
    pb = Z.make_problem(_p())
    pb.objective = 99
    assert Z.zeus_validate(pb) == Z.EINVAL
    assert Z.lib.zeus_validate(None) == Z.EINVAL


@pytest.mark.parametrize("unsup", [dict(dim=257)])
def test_validation_unsupported(Z, unsup):
    assert Z.zeus_validate(Z.make_problem(_p(**unsup))) == Z.EUNSUPPORTED


def test_workspace_bytes(Z):
    pb = Z.make_problem(_p(n=65536, dim=10))
    b = Z.zeus_workspace_bytes(pb)
    n, d = 65536, 10
    # swarm state x, v, px, pf plus the double-buffered block results of at
    # most 1024 blocks (value, key, index and a position each)
    assert 3 * 8 * n * d + 8 * n <= b <= 3 * 8 * n * d + 8 * n + 2 * 1024 * (d + 3) * 8 + 64 * 1024
    with pytest.raises(Z.ZeusError):
        Z.zeus_workspace_bytes(Z.make_problem(_p(dim=0)))


@pytest.mark.parametrize("n,d", [(100, 65), (700, 128), (5000, 200), (900, 208), (3000, 209),
                                 (3000, 256)])
def test_workspace_bytes_wide(Z, n, d):
    """Above 208 dimensions the workspace also holds one inverse-Hessian slot
    per resident block (at most 2048), d columns of the dimension rounded up to
    64; up to 208 the inverse Hessians stay on chip (registers, then registers
    and LDS)."""
    b = Z.zeus_workspace_bytes(Z.make_problem(_p(n=n, dim=d)))
    slots = min(n, 2048) if d > 208 else 0
    hs = 8 * slots * d * ((d + 63) // 64 * 64)
    swarm = 3 * 8 * n * d + 8 * n
    assert swarm + hs <= b <= swarm + hs + 2 * 1024 * (d + 3) * 8 + 64 * 1024


def test_context_without_device_is_a_clean_error(Z):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(Z.ZeusError) as e:
        Z.zeus_context_create(0)
    assert e.value.code in (Z.EHIP, Z.EINVAL)


def test_static_workspace_size_matches_header(Z):
    src = open(HEADER).read()
    m = re.search(r"#define ZEUS_STATIC_WORKSPACE_BYTES \(\(size_t\)(\d+) << (\d+)\)", src)
    assert m, "ZEUS_STATIC_WORKSPACE_BYTES not found"
    assert Z.STATIC_WORKSPACE_BYTES == int(m.group(1)) << int(m.group(2))
