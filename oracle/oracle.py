"""ctypes wrapper of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module.  It shares nothing with the GPU library; problems are
passed as plain dicts (see ``paper_2603_28770_amd.workloads``) and mapped to
the oracle's own struct here.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ZEUS_ORACLE_DIR names a directory holding other builds of both libraries
# (the sanitizer builds of build.build_sanitized)
_DIR = os.environ.get("ZEUS_ORACLE_DIR") or HERE
LIB_PATH = os.path.join(_DIR, "libzeus_oracle.so")
# the plain build: sums left to right, unfused row products and update, the C
# library's sin/cos/exp/log (see zeus_oracle.h)
LIB_PLAIN_PATH = os.path.join(_DIR, "libzeus_oracle_plain.so")

OBJECTIVES = {"rosenbrock": 0, "rastrigin": 1, "ackley": 2, "styblinski_tang": 3,
              "goldstein_price": 4, "sphere": 5, "quartic": 6, "user": 7}
MAXITER, CONVERGED, STOPPED, NONFINITE = 0, 1, 2, 3
TAG_X0, TAG_V0, TAG_R1, TAG_R2 = 0, 1, 2, 3


class _Problem(C.Structure):
    _fields_ = [("objective", C.c_int32), ("dim", C.c_int32), ("n", C.c_int64),
                ("lower", C.c_double), ("upper", C.c_double),
                ("iter_pso", C.c_int32), ("w", C.c_double), ("c1", C.c_double),
                ("c2", C.c_double), ("v_half", C.c_double),
                ("iter_bfgs", C.c_int32), ("iter_ls", C.c_int32),
                ("armijo_c", C.c_double), ("ls_shrink", C.c_double),
                ("grad_tol", C.c_double), ("seed", C.c_uint64),
                ("request_id", C.c_uint64), ("lbfgs_m", C.c_int32)]


class _Swarm(C.Structure):
    _fields_ = [("x", C.c_void_p), ("v", C.c_void_p), ("px", C.c_void_p),
                ("pf", C.c_void_p), ("gx", C.c_void_p), ("gf", C.c_double),
                ("gidx", C.c_int64), ("near_ties", C.c_int64)]


class _BfgsOut(C.Structure):
    _fields_ = [("x", C.c_void_p), ("f", C.c_void_p), ("iters", C.c_void_p),
                ("status", C.c_void_p), ("ls_trials", C.c_void_p),
                ("ls_fail", C.c_void_p), ("skips", C.c_void_p),
                ("resets", C.c_void_p), ("min_margin", C.c_void_p),
                ("tie_iter", C.c_void_p), ("trace", C.c_void_p),
                ("trace_len", C.c_int32)]


_libs = {}


def lib(plain=False):
    """The default build of the oracle, or with plain=True the plain build."""
    if plain not in _libs:
        path = LIB_PLAIN_PATH if plain else LIB_PATH
        if not os.path.exists(path):
            from oracle import build as _build
            _build.build()
        L = C.CDLL(path)
        L.zo_philox4x64_10.argtypes = [C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        L.zo_uniform.restype = C.c_double
        L.zo_uniform.argtypes = [C.c_uint64] * 6
        L.zo_f.restype = C.c_double
        L.zo_f.argtypes = [C.c_int, C.c_void_p, C.c_int]
        L.zo_grad.argtypes = [C.c_int, C.c_void_p, C.c_int, C.POINTER(C.c_double), C.c_void_p]
        L.zo_hrow_dot.restype = C.c_double
        L.zo_hrow_dot.argtypes = [C.c_void_p, C.c_void_p, C.c_int]
        L.zo_bfgs_update.restype = C.c_int
        L.zo_bfgs_update.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.zo_lbfgs_direction.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                         C.c_int, C.c_void_p]
        L.zo_line_search.restype = C.c_double
        L.zo_line_search.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_double, C.c_void_p,
                                     C.c_double, C.c_void_p, C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32)]
        L.zo_validate.restype = C.c_int
        L.zo_validate.argtypes = [C.POINTER(_Problem)]
        L.zo_pso.restype = C.c_int
        L.zo_pso.argtypes = [C.POINTER(_Problem), C.POINTER(_Swarm)]
        L.zo_bfgs.restype = C.c_int
        L.zo_bfgs.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_void_p, C.c_int64,
                              C.POINTER(_BfgsOut), C.c_int]
        L.zo_best.restype = C.c_int64
        L.zo_best.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]
        L.zo_max_threads.restype = C.c_int
        L.zo_lbfgs_push.restype = C.c_int
        L.zo_lbfgs_push.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int),
                                    C.c_int, C.c_void_p, C.c_void_p, C.c_int]
        for fn in ("zo_sin", "zo_cos", "zo_exp", "zo_log"):
            getattr(L, fn).restype = C.c_double
            getattr(L, fn).argtypes = [C.c_double]
        _libs[plain] = L
    return _libs[plain]


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def make_problem(p: dict) -> _Problem:
    """Map a workload dict to the oracle's struct (defaults are the paper's)."""
    return _Problem(
        objective=OBJECTIVES[p["objective"]], dim=int(p["dim"]), n=int(p["n"]),
        lower=float(p["lower"]), upper=float(p["upper"]),
        iter_pso=int(p.get("iter_pso", 0)), w=float(p.get("w", 0.5)),
        c1=float(p.get("c1", 1.2)), c2=float(p.get("c2", 1.5)),
        v_half=float(p.get("v_half", 0.0)), iter_bfgs=int(p.get("iter_bfgs", 100)),
        iter_ls=int(p.get("iter_ls", 20)), armijo_c=float(p.get("armijo_c", 0.3)),
        ls_shrink=float(p.get("ls_shrink", 0.5)), grad_tol=float(p.get("grad_tol", 1e-6)),
        seed=int(p.get("seed", 0)), request_id=int(p.get("request_id", 0)),
        lbfgs_m=int(p.get("lbfgs_m", 0)))


def philox(ctr, key):
    c = (C.c_uint64 * 4)(*[int(v) for v in ctr])
    k = (C.c_uint64 * 2)(*[int(v) for v in key])
    o = (C.c_uint64 * 4)()
    lib().zo_philox4x64_10(c, k, o)
    return [int(v) for v in o]


def uniform(seed, request_id, i, t, tag, j):
    return lib().zo_uniform(seed, request_id, i, t, tag, j)


def f(objective, x, plain=False):
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib(plain).zo_f(OBJECTIVES[objective], _ptr(x), x.size)


def grad(objective, x, plain=False):
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.empty_like(x)
    fv = C.c_double()
    lib(plain).zo_grad(OBJECTIVES[objective], _ptr(x), x.size, C.byref(fv), _ptr(g))
    return fv.value, g


def lbfgs_direction(S, Y, rho, g, plain=False):
    """Two-loop recursion p = -H g over the pairs in the rows of S, Y (oldest first)."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    p = np.empty_like(g)
    lib(plain).zo_lbfgs_direction(_ptr(S), _ptr(Y), _ptr(rho), int(rho.size), _ptr(g), g.size, _ptr(p))
    return p


def lbfgs_push(S, Y, rho, count, s_vec, y_vec, plain=False):
    """The pair window update (zo_lbfgs_push) in place on S, Y [m][d] and
    rho [m]; returns (new count, stored)."""
    cnt = C.c_int(int(count))
    s_vec = np.ascontiguousarray(s_vec, dtype=np.float64)
    y_vec = np.ascontiguousarray(y_vec, dtype=np.float64)
    ok = lib(plain).zo_lbfgs_push(_ptr(S), _ptr(Y), _ptr(rho), C.byref(cnt), S.shape[0],
                                  _ptr(s_vec), _ptr(y_vec), s_vec.size)
    return cnt.value, bool(ok)


def sin(x, plain=False):
    return lib(plain).zo_sin(float(x))


def cos(x, plain=False):
    return lib(plain).zo_cos(float(x))


def exp(x, plain=False):
    return lib(plain).zo_exp(float(x))


def hrow_dot(hrow, v, plain=False):
    """Row of H times v in the order of the BFGS matvecs (16-column fused
    multiply-add chains, block sums added pairwise; plain build: unfused,
    columns ascending)."""
    hrow = np.ascontiguousarray(hrow, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    return float(lib(plain).zo_hrow_dot(_ptr(hrow), _ptr(v), hrow.size))


def bfgs_update(H, s, y, plain=False):
    H = np.array(H, dtype=np.float64, order="C", copy=True)
    s = np.ascontiguousarray(s, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    applied = lib(plain).zo_bfgs_update(_ptr(H), _ptr(s), _ptr(y), s.size)
    return H, bool(applied)


def line_search(problem, x, f0, p, ddir, plain=False):
    pb = make_problem(problem)
    x = np.ascontiguousarray(x, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    xt = np.empty_like(x)
    tr, acc = C.c_int32(), C.c_int32()
    a = lib(plain).zo_line_search(C.byref(pb), _ptr(x), float(f0), _ptr(p), float(ddir), _ptr(xt),
                             C.byref(tr), C.byref(acc))
    return a, tr.value, bool(acc.value)


def validate(problem) -> bool:
    try:
        pb = make_problem(problem)
    except (KeyError, ValueError, OverflowError, TypeError):
        return False
    return lib().zo_validate(C.byref(pb)) == 0


def pso(problem, plain=False):
    pb = make_problem(problem)
    n, d = pb.n, pb.dim
    out = {k: np.empty((n, d)) for k in ("x", "v", "px")}
    out["pf"] = np.empty(n)
    out["gx"] = np.empty(d)
    sw = _Swarm(x=_ptr(out["x"]), v=_ptr(out["v"]), px=_ptr(out["px"]), pf=_ptr(out["pf"]),
                gx=_ptr(out["gx"]))
    rc = lib(plain).zo_pso(C.byref(pb), C.byref(sw))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    out["gf"], out["gidx"], out["near_ties"] = sw.gf, sw.gidx, sw.near_ties
    return out


def bfgs(problem, x0, idx=None, trace_len=0, nthreads=None, plain=False):
    pb = make_problem(problem)
    d = pb.dim
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        m = idx.size
    else:
        m = x0.shape[0]
    o = {"x": np.empty((m, d)), "f": np.empty(m), "iters": np.empty(m, np.int32),
         "status": np.empty(m, np.int32), "ls_trials": np.empty(m, np.int32),
         "ls_fail": np.empty(m, np.int32), "skips": np.empty(m, np.int32),
         "resets": np.empty(m, np.int32), "min_margin": np.empty(m),
         "tie_iter": np.empty(m, np.int32)}
    if trace_len > 0:
        o["trace"] = np.full((m, trace_len, d), np.nan)
    bo = _BfgsOut(x=_ptr(o["x"]), f=_ptr(o["f"]), iters=_ptr(o["iters"]),
                  status=_ptr(o["status"]), ls_trials=_ptr(o["ls_trials"]),
                  ls_fail=_ptr(o["ls_fail"]), skips=_ptr(o["skips"]), resets=_ptr(o["resets"]),
                  min_margin=_ptr(o["min_margin"]), tie_iter=_ptr(o["tie_iter"]),
                  trace=_ptr(o.get("trace")), trace_len=int(trace_len))
    nt = nthreads if nthreads else lib(plain).zo_max_threads()
    rc = lib(plain).zo_bfgs(C.byref(pb), _ptr(x0), _ptr(idx), m, C.byref(bo), int(nt))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    o["threads"] = nt
    return o


ST_CONVERGED, ST_STOPPED = 1, 2


def bfgs_required(problem, x0, required_c, nthreads=None, plain=False):
    """Alg. 10's early stop (required_c starts converged), read iteration-
    synchronously: K* is the iteration at which the required_c-th start
    converges (the required_c-th smallest iteration count among converged
    starts).  Every start still running at K* ends there: its result is its
    iterate after K* steps, status STOPPED.  Starts that ended at K* or before
    keep their results.  With fewer than required_c convergences nothing
    stops early.  Returns the per-start results and K* (None if no stop)."""
    full = bfgs(problem, x0, nthreads=nthreads, plain=plain)
    conv = np.sort(full["iters"][full["status"] == ST_CONVERGED])
    if required_c <= 0 or conv.size < required_c:
        return full, None
    kstar = int(conv[required_c - 1])
    late = np.flatnonzero(full["iters"] > kstar)
    if late.size:
        cut = bfgs(dict(problem, iter_bfgs=kstar), x0, idx=late, nthreads=nthreads, plain=plain)
        for k in ("x", "f", "iters", "ls_trials", "skips", "resets"):
            full[k][late] = cut[k]
        full["status"][late] = ST_STOPPED
    return full, kstar


def best(fvals, status):
    fvals = np.ascontiguousarray(fvals, dtype=np.float64)
    status = np.ascontiguousarray(status, dtype=np.int32)
    nc = C.c_int64()
    b = lib().zo_best(_ptr(fvals), _ptr(status), fvals.size, C.byref(nc))
    return int(b), int(nc.value)


def max_threads():
    return lib().zo_max_threads()


def minimize(problem, idx=None, trace_len=0, nthreads=None, plain=False):
    """PSO then BFGS from every start (or the starts listed in idx)."""
    sw = pso(problem, plain=plain)
    r = bfgs(problem, sw["x"], idx=idx, trace_len=trace_len, nthreads=nthreads, plain=plain)
    b, nc = best(r["f"], r["status"])
    r["best_index"] = b if idx is None or b < 0 else int(np.asarray(idx)[b])
    r["best_f"] = float(r["f"][b]) if b >= 0 else float("nan")
    r["n_converged"] = nc
    r["swarm"] = sw
    return r


class View:
    """This module's functions bound to one build of the oracle: the default
    build (plain=False) or the plain build (plain=True)."""

    def __init__(self, plain=False):
        self.plain = bool(plain)

    def __getattr__(self, name):
        import functools
        import inspect
        obj = globals()[name]
        if callable(obj) and not isinstance(obj, type):
            try:
                if "plain" in inspect.signature(obj).parameters:
                    return functools.partial(obj, plain=self.plain)
            except (TypeError, ValueError):
                pass
        return obj

    def lib(self):
        return lib(self.plain)
