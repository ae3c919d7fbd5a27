"""The allocation-free entry point (zeus_minimize_async_static) against the
ordinary asynchronous one (zeus_minimize_async with a caller workspace),
through the C ABI: the same kernels run either way, so every output must be
bit-identical.  Two calls in a row on the same stream, the second with a
smaller problem (the static workspace keeps the first call's contents), then
the block kernels (inverse Hessians on chip up to dim 208, in the workspace
above), and the clear error for a problem larger than the static
workspace."""
import numpy as np
import pytest

from paper_2603_28770_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Z():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_28770_amd import zeus
    return zeus


@pytest.fixture(scope="module")
def ctx(Z):
    c = Z.zeus_context_create(0)
    yield c
    Z.zeus_context_destroy(c)


KEYS = ("f", "x", "iters", "status", "ls_trials", "skips", "resets", "seeds", "pso_v", "pso_px", "pso_pf",
        "pso_best_x", "trace")


def _both(Z, ctx, p, stream):
    a = Z.DeviceSolve(p, trace_len=3, pso_state=True)
    a.enqueue(ctx, stream.cuda_stream)
    stream.synchronize()
    ra = a.host()
    b = Z.DeviceSolve(p, trace_len=3, pso_state=True)
    b.enqueue_static(ctx, stream.cuda_stream)
    stream.synchronize()
    rb = b.host()
    return ra, rb


def _same(ra, rb):
    for k in KEYS:
        assert np.array_equal(ra[k], rb[k], equal_nan=True), k
    assert ra["summary"] == rb["summary"]


def test_static_workspace_two_calls_then_smaller(Z, ctx):
    import torch
    s = torch.cuda.Stream()
    big = W.RASTRIGIN_D10                       # about 16 MB of workspace
    small = W.problem(name="rosenbrock_d7", objective="rosenbrock", dim=7, n=3000, lower=-2.0,
                      upper=2.0, iter_pso=3, iter_bfgs=300, seed=9)
    assert Z.zeus_workspace_bytes(Z.make_problem(big)) <= Z.STATIC_WORKSPACE_BYTES
    for p in (big, small):
        print(f"\n[static] {p['name']} n={p['n']} d={p['dim']}", flush=True)
        ra, rb = _both(Z, ctx, p, s)
        _same(ra, rb)


@pytest.mark.parametrize("dim", [100, 150, 220], ids=["registers", "registers_lds", "slots"])
def test_static_workspace_with_inverse_hessian_slots(Z, ctx, dim):
    """The block kernels: H in registers (d = 100), in registers and LDS
    (d = 150) and in device-memory slots carved from the workspace (d = 220)."""
    import torch
    s = torch.cuda.Stream()
    p = W.problem(name=f"styblinski_d{dim}", objective="styblinski_tang", dim=dim, n=40,
                  lower=-5.0, upper=5.0, iter_pso=2, iter_bfgs=150, seed=3)
    assert Z.zeus_workspace_bytes(Z.make_problem(p)) <= Z.STATIC_WORKSPACE_BYTES
    print(f"\n[static] {p['name']}", flush=True)
    ra, rb = _both(Z, ctx, p, s)
    _same(ra, rb)


def test_static_workspace_too_small_is_a_clean_error(Z, ctx):
    p = W.ROSENBROCK_D50                        # about 160 MB of workspace
    assert Z.zeus_workspace_bytes(Z.make_problem(p)) > Z.STATIC_WORKSPACE_BYTES
    d = Z.DeviceSolve(W.scaled(p, 8))           # outputs only need to be valid pointers
    with pytest.raises(Z.ZeusError) as e:
        Z.zeus_minimize_async_static(ctx, p, d.result, 0)
    assert e.value.code == Z.ENOMEM
    assert "static workspace" in str(e.value)
