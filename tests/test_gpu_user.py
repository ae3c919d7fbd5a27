"""User-defined objectives on the GPU (compiled at run time with hipRTC)
against the oracle running the same source compiled for the CPU: swarm seeds
and every start's f, x, iterations, status and line-search trials bit for
bit, for one to four requests per call (a Goldstein-Price batch), every lane
count from 4 to 64, trigonometric, logarithmic and exponential user code
(a binned Poisson likelihood fit), BFGS on the on-chip block kernels at
d = 100 and 150, L-BFGS from d = 5 to d = 200 (one, two and four coordinates
per lane), and early stop; mixed precision (the user code run on the FP32
number types) against the FP64 oracle, with the bars of the built-in
objectives' mixed mode; plus the refusals."""
import numpy as np
import pytest

from oracle import user as OU
from paper_2603_28770_amd import user_objectives as UO
from paper_2603_28770_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("f", "x", "iters", "status", "ls_trials", "skips", "resets")


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


def _p(d, n, lo, hi, seed, **kw):
    return W.problem(objective="user", dim=d, n=n, lower=lo, upper=hi, seed=seed,
                     iter_pso=kw.pop("iter_pso", 5), iter_bfgs=kw.pop("iter_bfgs", 300), **kw)


CASES = [
    ("rosenbrock_d2", UO.ROSENBROCK, [_p(2, 512, -5.0, 5.0, 1)]),
    ("rosenbrock_d9", UO.ROSENBROCK, [_p(9, 300, -2.0, 2.0, 2)]),
    ("goldstein_price_batch", UO.GOLDSTEIN_PRICE,
     [_p(2, 256, -2.0, 2.0, s, request_id=s) for s in range(4)]),
    ("rastrigin_d5", UO.RASTRIGIN, [_p(5, 400, -5.12, 5.12, 3, iter_pso=10)]),
    ("chain_log_d20", UO.CHAIN_LOG, [_p(20, 256, -2.0, 2.0, 4)]),
    ("chain_log_d40", UO.CHAIN_LOG, [_p(40, 128, -2.0, 2.0, 5, iter_bfgs=200)]),
    ("poisson_fit_d4", "poisson", [_p(4, 512, 0.0, 10.0, 6, iter_pso=10, iter_bfgs=500)]),
    # L-BFGS: one coordinate per lane, then two and four per lane (d > 64)
    ("chain_log_d20_lbfgs", UO.CHAIN_LOG, [_p(20, 256, -2.0, 2.0, 11, lbfgs_m=5)]),
    ("rastrigin_d5_lbfgs", UO.RASTRIGIN, [_p(5, 300, -5.12, 5.12, 12, lbfgs_m=3)]),
    ("chain_log_d100_lbfgs", UO.CHAIN_LOG, [_p(100, 96, -2.0, 2.0, 13, lbfgs_m=6, iter_bfgs=150)]),
    ("rosenbrock_d200_lbfgs", UO.ROSENBROCK,
     [_p(200, 64, -2.0, 2.0, 14, iter_pso=2, lbfgs_m=8, iter_bfgs=150)]),
    # BFGS above 64 dimensions: one block per start, H in registers (d <= 128),
    # then in registers and LDS (d <= 208)
    ("chain_log_d100", UO.CHAIN_LOG, [_p(100, 48, -2.0, 2.0, 15, iter_pso=2, iter_bfgs=120)]),
    ("rosenbrock_d150", UO.ROSENBROCK, [_p(150, 32, -2.0, 2.0, 16, iter_pso=2, iter_bfgs=150)]),
]


@pytest.fixture(scope="module")
def compiled(Z, ctx):
    objs = {}
    yield lambda src: objs.setdefault(src, Z.zeus_objective_compile(ctx, src))
    for h in objs.values():
        Z.zeus_objective_destroy(h)


@pytest.mark.parametrize("name,src,problems", CASES, ids=[c[0] for c in CASES])
def test_user_objective_matches_oracle(Z, ctx, compiled, oracle_mod, name, src, problems):
    src = UO.poisson_fit_source() if src == "poisson" else src
    print(f"\n[user] {name}: {len(problems)} request(s), d = {problems[0]['dim']}", flush=True)
    obj = compiled(src)
    outs = Z.zeus_minimize_user(ctx, obj, problems, pso_state=True)
    OU.use(src, oracle_mod.lib())
    for p, g in zip(problems, outs):
        sw = oracle_mod.pso(p)
        assert np.array_equal(g["seeds"], sw["x"])
        o = oracle_mod.bfgs(p, sw["x"])
        for k in KEYS:
            assert np.array_equal(g[k], o[k], equal_nan=True), (name, k)
        print(f"[user]   converged {int(np.sum(o['status'] == 1))}/{p['n']}, "
              f"best f {np.nanmin(o['f']):.6g}", flush=True)


def test_user_rosenbrock_bench_size_sample(Z, ctx, compiled, oracle_mod):
    """The user-code Rosenbrock bench problem at full size (d = 50, 131,072
    starts, the launch the bench times): every swarm seed equals the oracle
    swarm's, and 32 strided starts' results equal the oracle's BFGS from those
    seeds."""
    p = W.USER_ROSENBROCK_D50
    print(f"\n[user] rosenbrock d = {p['dim']}, n = {p['n']} (bench size)", flush=True)
    g = Z.zeus_minimize_user(ctx, compiled(UO.ROSENBROCK), [p], pso_state=True)[0]
    OU.use(UO.ROSENBROCK, oracle_mod.lib())
    sw = oracle_mod.pso(p)
    assert np.array_equal(g["seeds"], sw["x"])
    idx = W.strided_subset(p["n"], 32)
    o = oracle_mod.bfgs(p, sw["x"], idx=idx)
    for k in KEYS:
        assert np.array_equal(g[k][idx], o[k], equal_nan=True), k
    print(f"[user]   sample converged {int(np.sum(o['status'] == 1))}/{idx.size}", flush=True)


def test_user_objective_early_stop(Z, ctx, compiled, oracle_mod):
    p = _p(20, 256, -2.0, 2.0, 8)
    print("\n[user] chain_log_d20 with required_converged = 10", flush=True)
    g = Z.zeus_minimize_user(ctx, compiled(UO.CHAIN_LOG), [dict(p, required_converged=10)])[0]
    OU.use(UO.CHAIN_LOG, oracle_mod.lib())
    o, kstar = oracle_mod.bfgs_required(p, oracle_mod.pso(p)["x"], 10)
    for k in KEYS:
        assert np.array_equal(g[k], o[k], equal_nan=True), k
    assert np.sum(g["status"] == Z.ST_STOPPED) > 0


def test_poisson_fit_recovers_the_spectrum(Z, ctx, compiled, oracle_mod):
    """A sanity check of the example, not parity: the best converged start is
    a maximum-likelihood fit, at least as likely as the generating parameters
    (which are strongly correlated, so the fit may sit far from them in
    parameter space), and its expected counts describe the spectrum within
    the Poisson errors of every bin."""
    src = UO.poisson_fit_source()
    g = Z.zeus_minimize_user(ctx, compiled(src),
                             [_p(4, 2048, 0.0, 10.0, 9, iter_pso=10, iter_bfgs=500)])[0]
    b = int(np.nanargmin(np.where(g["status"] == 1, g["f"], np.nan)))
    OU.use(src, oracle_mod.lib())
    assert g["f"][b] <= oracle_mod.f("user", np.array(UO.POISSON_TRUE, dtype=np.float64))
    _, l1, lx, n = UO.poisson_histogram()

    def mu(t):
        return np.exp(t[0] + t[1] * l1 - (t[2] + t[3] * lx) * lx)

    m_fit, m_true = mu(g["x"][b]), mu(UO.POISSON_TRUE)
    assert np.all(np.abs(m_fit - m_true) <= 4.0 * np.sqrt(m_true) + 1.0)


MIXED_CASES = [
    ("rosenbrock_d9", UO.ROSENBROCK, _p(9, 300, -2.0, 2.0, 2, iter_bfgs=1000), 0.8),
    ("rastrigin_d5", UO.RASTRIGIN, _p(5, 400, -5.12, 5.12, 3, iter_pso=10, iter_bfgs=500), 0.6),
    ("goldstein_price_d2", UO.GOLDSTEIN_PRICE, _p(2, 512, -2.0, 2.0, 1, iter_bfgs=500), 0.8),
    ("poisson_fit_d4", "poisson", _p(4, 512, 0.0, 10.0, 6, iter_pso=10, iter_bfgs=500), 0.5),
    ("chain_log_d20_lbfgs", UO.CHAIN_LOG, _p(20, 256, -2.0, 2.0, 11, lbfgs_m=5, iter_bfgs=500), 0.8),
    ("chain_log_d100_lbfgs", UO.CHAIN_LOG,
     _p(100, 96, -2.0, 2.0, 13, lbfgs_m=6, iter_pso=2, iter_bfgs=400), 0.6),
    # one block per start: H in registers, then in registers and LDS
    ("chain_log_d100", UO.CHAIN_LOG, _p(100, 96, -2.0, 2.0, 15, iter_pso=2, iter_bfgs=400), 0.6),
    ("rosenbrock_d150", UO.ROSENBROCK, _p(150, 32, -2.0, 2.0, 16, iter_pso=2, iter_bfgs=2000), 0.6),
]


@pytest.mark.parametrize("name,src,p,min_same", MIXED_CASES, ids=[c[0] for c in MIXED_CASES])
def test_user_mixed_against_fp64_oracle(Z, ctx, compiled, oracle_mod, name, src, p, min_same):
    """Mixed precision with user code: the swarm is FP64 and matches bit for
    bit; the reported f is the FP64 value of the user code at the returned x;
    a converged start's FP64 gradient norm is below Theta (the convergence
    test is taken in FP64 after the escalation); most starts end at the
    oracle's minimum to within FP32 noise (relative 1e-4 in f), and the
    success rates (f within 1e-4 of the best FP64 value) agree: within 0.01,
    or, with few starts, within three times the spread that the starts ending
    elsewhere than the oracle's give by themselves."""
    src = UO.poisson_fit_source() if src == "poisson" else src
    pm = dict(p, precision="mixed", grad_tol=1e-4)
    print(f"\n[user mixed] {name}: d = {p['dim']}, n = {p['n']}", flush=True)
    g = Z.zeus_minimize_user(ctx, compiled(src), [pm], pso_state=True)[0]
    OU.use(src, oracle_mod.lib())
    sw = oracle_mod.pso(pm)
    assert np.array_equal(g["seeds"], sw["x"]) and np.array_equal(g["pso_pf"], sw["pf"])
    o = oracle_mod.bfgs(pm, sw["x"])
    for i in range(0, p["n"], max(1, p["n"] // 25)):
        if np.isfinite(g["f"][i]):
            assert g["f"][i] == oracle_mod.f("user", g["x"][i])
    conv = np.flatnonzero(g["status"] == 1)
    for i in conv[:: max(1, conv.size // 25)]:
        _, gr = oracle_mod.grad("user", g["x"][i])
        assert np.linalg.norm(gr) < 1.01 * pm["grad_tol"], i
    fs = np.maximum(1.0, np.abs(o["f"]))
    same = np.abs(g["f"] - o["f"]) / fs <= 1e-4
    best = min(np.nanmin(o["f"]), np.nanmin(g["f"]))
    tol = 1e-4 * max(1.0, abs(best))
    rg, ro = np.mean(g["f"] - best < tol), np.mean(o["f"] - best < tol)
    print(f"[user mixed]   same minimum {same.mean():.3f}; converged gpu "
          f"{np.mean(g['status'] == 1):.3f} oracle {np.mean(o['status'] == 1):.3f}; "
          f"success gpu {rg:.4f} oracle {ro:.4f}", flush=True)
    assert same.mean() >= min_same
    # a start that ends elsewhere than the oracle's succeeds or fails on its
    # own: from those starts alone the rates differ by about sqrt(q / n), q
    # their share
    assert abs(rg - ro) <= max(0.01, 3.0 * np.sqrt((1.0 - same.mean()) / p["n"]))


def test_user_refusals(Z, ctx, compiled):
    obj = compiled(UO.ROSENBROCK)
    for bad, code in ((dict(dim=209), Z.EUNSUPPORTED), (dict(dim=209, precision="mixed"), Z.EUNSUPPORTED),
                      (dict(dim=257, lbfgs_m=4), Z.EUNSUPPORTED), (dict(lbfgs_m=9), Z.EUNSUPPORTED),
                      (dict(objective="rosenbrock"), Z.EINVAL)):
        with pytest.raises(Z.ZeusError) as e:
            Z.zeus_minimize_user(ctx, obj, [dict(_p(3, 16, -1.0, 1.0, 0), **bad)])
        assert e.value.code == code, bad
    with pytest.raises(Z.ZeusError) as e:
        Z.zeus_minimize(ctx, _p(3, 16, -1.0, 1.0, 0))
    assert e.value.code == Z.EINVAL
    with pytest.raises(Z.ZeusError) as e:
        Z.zeus_objective_compile(ctx, "this is not C++")
    assert e.value.code == Z.EINVAL
