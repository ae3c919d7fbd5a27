"""Thin ctypes binding of libzeus.so (the C ABI in include/zeus.h).

The entry points keep their C names; this module only marshals arguments.
Every step of the method runs in the HIP kernels of libzeus.so; there is no
fallback: if the library is missing, importing this module raises.

PyTorch (imported first, so that one HIP runtime serves both) supplies device
memory and streams for the asynchronous entry point.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ZEUS_LIB names another build of the same library (e.g. to compare builds).
LIB_PATH = os.environ.get("ZEUS_LIB") or os.path.join(HERE, "libzeus.so")

ABI_VERSION = 2
OK, NOT_READY, EINVAL, ENOMEM, EHIP, EUNSUPPORTED, ECANCELLED, ETIMEOUT = 0, 1, -1, -2, -3, -4, -5, -6
OBJECTIVES = {"rosenbrock": 0, "rastrigin": 1, "ackley": 2, "styblinski_tang": 3,
              "goldstein_price": 4, "sphere": 5, "quartic": 6, "user": 7}
PRECISIONS = {"fp64": 0, "mixed": 1}
ST_MAXITER, ST_CONVERGED, ST_STOPPED, ST_NONFINITE = 0, 1, 2, 3

# Symbols declared in include/zeus.h.
EXPORTS = ("zeus_abi_version", "zeus_version", "zeus_last_error", "zeus_validate",
           "zeus_workspace_bytes", "zeus_context_create", "zeus_context_destroy",
           "zeus_context_set_profiling", "zeus_context_get_profile", "zeus_minimize",
           "zeus_minimize_batch", "zeus_minimize_async", "zeus_minimize_async_static",
           "zeus_server_create", "zeus_server_create_emulated", "zeus_server_request_bytes",
           "zeus_server_submit", "zeus_server_wait", "zeus_server_cancel", "zeus_server_destroy",
           "zeus_plan_workspace_bytes", "zeus_plan_create", "zeus_plan_launch", "zeus_plan_destroy",
           "zeus_objective_compile", "zeus_objective_check", "zeus_objective_destroy",
           "zeus_minimize_user")


class zeus_problem(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("objective", C.c_int32), ("dim", C.c_int32),
                ("precision", C.c_int32), ("n_starts", C.c_int64), ("lower", C.c_double),
                ("upper", C.c_double), ("iter_pso", C.c_int32), ("iter_bfgs", C.c_int32),
                ("iter_ls", C.c_int32), ("lbfgs_m", C.c_int32), ("w", C.c_double),
                ("c1", C.c_double), ("c2", C.c_double), ("v_half", C.c_double),
                ("armijo_c", C.c_double), ("ls_shrink", C.c_double), ("grad_tol", C.c_double),
                ("required_converged", C.c_int64), ("seed", C.c_uint64),
                ("request_id", C.c_uint64)]


class zeus_summary(C.Structure):
    _fields_ = [("best_index", C.c_int64), ("best_f", C.c_double), ("n_converged", C.c_int64),
                ("n_nonfinite", C.c_int64), ("total_iters", C.c_int64),
                ("total_ls_trials", C.c_int64), ("pso_best_index", C.c_int64),
                ("pso_best_f", C.c_double)]


class zeus_result(C.Structure):
    _fields_ = [("f", C.c_void_p), ("x", C.c_void_p), ("iters", C.c_void_p),
                ("status", C.c_void_p), ("ls_trials", C.c_void_p), ("seeds", C.c_void_p),
                ("pso_v", C.c_void_p), ("pso_px", C.c_void_p), ("pso_pf", C.c_void_p),
                ("pso_best_x", C.c_void_p), ("trace", C.c_void_p), ("trace_len", C.c_int32),
                ("reserved0", C.c_int32), ("summary", C.c_void_p), ("skips", C.c_void_p),
                ("resets", C.c_void_p)]


class zeus_profile(C.Structure):
    _fields_ = [("pso_ms", C.c_double), ("bfgs_ms", C.c_double), ("reduce_ms", C.c_double),
                ("pso_launches", C.c_int64), ("bfgs_launches", C.c_int64),
                ("reduce_launches", C.c_int64)]


class zeus_request_times(C.Structure):
    _fields_ = [("t_submit_ns", C.c_uint64), ("t_admit_ns", C.c_uint64), ("t_done_ns", C.c_uint64)]


class zeus_emulation(C.Structure):
    _fields_ = [("swarm_ns", C.c_uint64), ("step_ns", C.c_uint64), ("start_ns", C.c_uint64),
                ("finish_ns", C.c_uint64), ("resident_starts", C.c_int64)]


class ZeusError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"zeus error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2603_28770_amd.build` (no fallback exists)")
    try:  # share torch's HIP runtime when torch is present
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    L.zeus_abi_version.restype = C.c_uint32
    L.zeus_version.restype = C.c_char_p
    L.zeus_last_error.restype = C.c_char_p
    L.zeus_validate.argtypes = [P(zeus_problem)]
    L.zeus_workspace_bytes.argtypes = [P(zeus_problem), P(C.c_size_t)]
    L.zeus_context_create.argtypes = [C.c_int, P(C.c_void_p)]
    L.zeus_context_destroy.argtypes = [C.c_void_p]
    L.zeus_context_set_profiling.argtypes = [C.c_void_p, C.c_int]
    L.zeus_context_get_profile.argtypes = [C.c_void_p, P(zeus_profile)]
    L.zeus_minimize.argtypes = [C.c_void_p, P(zeus_problem), P(zeus_result)]
    L.zeus_minimize_batch.argtypes = [C.c_void_p, P(zeus_problem), C.c_int32, P(zeus_result)]
    L.zeus_minimize_async.argtypes = [C.c_void_p, P(zeus_problem), C.c_void_p, C.c_size_t,
                                      P(zeus_result), C.c_void_p]
    L.zeus_minimize_async_static.argtypes = [C.c_void_p, P(zeus_problem), P(zeus_result),
                                             C.c_void_p]
    L.zeus_server_create.argtypes = [C.c_void_p, C.c_size_t, P(C.c_void_p)]
    L.zeus_server_create_emulated.argtypes = [C.c_size_t, P(zeus_emulation), P(C.c_void_p)]
    L.zeus_server_request_bytes.argtypes = [P(zeus_problem), P(zeus_result), P(C.c_size_t)]
    L.zeus_server_submit.argtypes = [C.c_void_p, P(zeus_problem), P(zeus_result), P(C.c_uint64)]
    L.zeus_server_wait.argtypes = [C.c_void_p, C.c_uint64, C.c_int64, P(zeus_request_times)]
    L.zeus_server_cancel.argtypes = [C.c_void_p, C.c_uint64]
    L.zeus_server_destroy.argtypes = [C.c_void_p]
    L.zeus_plan_workspace_bytes.argtypes = [P(zeus_problem), C.c_int32, P(C.c_size_t)]
    L.zeus_plan_create.argtypes = [C.c_void_p, P(zeus_problem), C.c_int32, C.c_void_p, C.c_size_t,
                                   P(zeus_result), P(C.c_void_p)]
    L.zeus_plan_launch.argtypes = [C.c_void_p, C.c_void_p]
    L.zeus_plan_destroy.argtypes = [C.c_void_p]
    L.zeus_objective_compile.argtypes = [C.c_void_p, C.c_char_p, P(C.c_void_p)]
    L.zeus_objective_check.argtypes = [C.c_char_p]
    L.zeus_objective_destroy.argtypes = [C.c_void_p]
    L.zeus_minimize_user.argtypes = [C.c_void_p, C.c_void_p, P(zeus_problem), C.c_int32, P(zeus_result)]
    for name in EXPORTS:
        if name not in ("zeus_abi_version", "zeus_version", "zeus_last_error"):
            getattr(L, name).restype = C.c_int
    return L


lib = _load()


def _check(code):
    if code != OK:
        raise ZeusError(code, lib.zeus_last_error().decode())
    return code


def make_problem(p: dict) -> zeus_problem:
    """Map a workload dict to zeus_problem (defaults are the paper's)."""
    return zeus_problem(
        abi_version=ABI_VERSION, objective=OBJECTIVES[p["objective"]], dim=int(p["dim"]),
        precision=PRECISIONS[p.get("precision", "fp64")], n_starts=int(p["n"]),
        lower=float(p["lower"]), upper=float(p["upper"]), iter_pso=int(p.get("iter_pso", 0)),
        iter_bfgs=int(p.get("iter_bfgs", 100)), iter_ls=int(p.get("iter_ls", 20)), lbfgs_m=int(p.get("lbfgs_m", 0)),
        w=float(p.get("w", 0.5)), c1=float(p.get("c1", 1.2)), c2=float(p.get("c2", 1.5)),
        v_half=float(p.get("v_half", 0.0)), armijo_c=float(p.get("armijo_c", 0.3)),
        ls_shrink=float(p.get("ls_shrink", 0.5)), grad_tol=float(p.get("grad_tol", 1e-6)),
        required_converged=int(p.get("required_converged", 0)), seed=int(p.get("seed", 0)),
        request_id=int(p.get("request_id", 0)))


# ---- C entry points under their own names --------------------------------------

def zeus_abi_version() -> int:
    return lib.zeus_abi_version()


def zeus_version() -> str:
    return lib.zeus_version().decode()


def zeus_last_error() -> str:
    return lib.zeus_last_error().decode()


def zeus_validate(problem: zeus_problem) -> int:
    return lib.zeus_validate(C.byref(problem))


def zeus_workspace_bytes(problem: zeus_problem) -> int:
    b = C.c_size_t()
    _check(lib.zeus_workspace_bytes(C.byref(problem), C.byref(b)))
    return b.value


def zeus_context_create(device: int = 0) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib.zeus_context_create(int(device), C.byref(h)))
    return h


def zeus_context_destroy(ctx) -> None:
    _check(lib.zeus_context_destroy(ctx))


def zeus_context_set_profiling(ctx, enabled: bool) -> None:
    _check(lib.zeus_context_set_profiling(ctx, 1 if enabled else 0))


def zeus_context_get_profile(ctx) -> dict:
    p = zeus_profile()
    _check(lib.zeus_context_get_profile(ctx, C.byref(p)))
    return {k: getattr(p, k) for k, _ in zeus_profile._fields_}


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p).value


def _host_outputs(pb, trace_len, pso_state, ls_trials):
    n, d = pb.n_starts, pb.dim
    o = {"f": np.full(n, np.nan), "x": np.empty((n, d)), "iters": np.empty(n, np.int32),
         "status": np.empty(n, np.int32)}
    if ls_trials:  # the per-start counters: line-search trials, update skips, direction resets
        o["ls_trials"] = np.empty(n, np.int32)
        o["skips"] = np.empty(n, np.int32)
        o["resets"] = np.empty(n, np.int32)
    if pso_state:
        o.update(seeds=np.empty((n, d)), pso_v=np.empty((n, d)), pso_px=np.empty((n, d)),
                 pso_pf=np.empty(n), pso_best_x=np.empty(d))
    if trace_len:
        o["trace"] = np.empty((n, trace_len, d))
    s = zeus_summary()
    r = zeus_result(f=_np_ptr(o["f"]), x=_np_ptr(o["x"]), iters=_np_ptr(o["iters"]),
                    status=_np_ptr(o["status"]), ls_trials=_np_ptr(o.get("ls_trials")),
                    seeds=_np_ptr(o.get("seeds")), pso_v=_np_ptr(o.get("pso_v")),
                    pso_px=_np_ptr(o.get("pso_px")), pso_pf=_np_ptr(o.get("pso_pf")),
                    pso_best_x=_np_ptr(o.get("pso_best_x")), trace=_np_ptr(o.get("trace")),
                    trace_len=int(trace_len), reserved0=0,
                    summary=C.cast(C.pointer(s), C.c_void_p).value,
                    skips=_np_ptr(o.get("skips")), resets=_np_ptr(o.get("resets")))
    return o, s, r


def _summary_dict(s):
    return {k: getattr(s, k) for k, _ in zeus_summary._fields_}


def zeus_minimize(ctx, problem, *, trace_len=0, pso_state=False, ls_trials=True) -> dict:
    """Blocking solve; returns host numpy arrays."""
    pb = problem if isinstance(problem, zeus_problem) else make_problem(problem)
    o, s, r = _host_outputs(pb, trace_len, pso_state, ls_trials)
    _check(lib.zeus_minimize(ctx, C.byref(pb), C.byref(r)))
    o["summary"] = _summary_dict(s)
    return o


def _solve_list(call, problems, trace_len, pso_state, ls_trials) -> list:
    pbs = (zeus_problem * len(problems))(
        *[p if isinstance(p, zeus_problem) else make_problem(p) for p in problems])
    outs, sums = [], []
    res = (zeus_result * len(problems))()
    for k in range(len(problems)):
        o, s, r = _host_outputs(pbs[k], trace_len, pso_state, ls_trials)
        outs.append(o)
        sums.append(s)
        res[k] = r
    _check(call(pbs, len(problems), res))
    for o, s in zip(outs, sums):
        o["summary"] = _summary_dict(s)
    return outs


def zeus_minimize_batch(ctx, problems, *, trace_len=0, pso_state=False, ls_trials=True) -> list:
    """Blocking solve of a list of problems (dicts or zeus_problem)."""
    return _solve_list(lambda p, n, r: lib.zeus_minimize_batch(ctx, p, n, r), problems, trace_len,
                       pso_state, ls_trials)


def zeus_objective_check(source: str) -> None:
    """Compiles a user objective's source for gfx950 without loading it
    (raises ZeusError with the compiler's messages)."""
    _check(lib.zeus_objective_check(source.encode()))


def zeus_objective_compile(ctx, source: str):
    """Compiles and loads a user objective; returns its handle."""
    h = C.c_void_p()
    _check(lib.zeus_objective_compile(ctx, source.encode(), C.byref(h)))
    return h


def zeus_objective_destroy(obj) -> None:
    _check(lib.zeus_objective_destroy(obj))


def zeus_minimize_user(ctx, obj, problems, *, trace_len=0, pso_state=False, ls_trials=True) -> list:
    """Blocking solve of problems (objective "user") of a compiled user objective."""
    if isinstance(problems, (dict, zeus_problem)):
        problems = [problems]
    return _solve_list(lambda p, n, r: lib.zeus_minimize_user(ctx, obj, p, n, r), problems, trace_len,
                       pso_state, ls_trials)


def zeus_minimize_async(ctx, problem, workspace_ptr: int, workspace_bytes: int,
                        result: zeus_result, stream_ptr: int = 0) -> None:
    """Enqueue a solve with caller-owned device memory (e.g. torch tensors)."""
    pb = problem if isinstance(problem, zeus_problem) else make_problem(problem)
    _check(lib.zeus_minimize_async(ctx, C.byref(pb), C.c_void_p(workspace_ptr),
                                   C.c_size_t(workspace_bytes), C.byref(result),
                                   C.c_void_p(stream_ptr) if stream_ptr else None))


# ZEUS_STATIC_WORKSPACE_BYTES of zeus.h: the largest workspace the
# allocation-free entry point serves.
STATIC_WORKSPACE_BYTES = 64 << 20


def zeus_minimize_async_static(ctx, problem, result: zeus_result, stream_ptr: int = 0) -> None:
    """Enqueue a solve into caller-owned device outputs with the library's
    fixed device workspace (no device allocation)."""
    pb = problem if isinstance(problem, zeus_problem) else make_problem(problem)
    _check(lib.zeus_minimize_async_static(ctx, C.byref(pb), C.byref(result),
                                          C.c_void_p(stream_ptr) if stream_ptr else None))


class Server:
    """A zeus_server: submit problems from any thread, wait for their results.

    The host arrays of each submitted request are kept here until it is waited
    for."""

    def __init__(self, ctx, budget_bytes: int, _emulation=None):
        self.h = C.c_void_p()
        if _emulation is None:
            _check(lib.zeus_server_create(ctx, C.c_size_t(int(budget_bytes)), C.byref(self.h)))
        else:
            _check(lib.zeus_server_create_emulated(C.c_size_t(int(budget_bytes)),
                                                   C.byref(_emulation), C.byref(self.h)))
        self._live = {}

    @classmethod
    def emulated(cls, budget_bytes: int, *, swarm_ns: int, step_ns: int, start_ns: int,
                 finish_ns: int, resident_starts: int) -> "Server":
        """zeus_server_create_emulated: the server's scheduling with no GPU
        (modelled times, placeholder results)."""
        emu = zeus_emulation(swarm_ns=swarm_ns, step_ns=step_ns, start_ns=start_ns,
                             finish_ns=finish_ns, resident_starts=resident_starts)
        return cls(None, budget_bytes, _emulation=emu)

    @staticmethod
    def request_bytes(problem, *, trace_len=0, pso_state=False, ls_trials=True) -> int:
        """zeus_server_request_bytes for a request with these outputs."""
        pb = problem if isinstance(problem, zeus_problem) else make_problem(problem)
        _, _, r = _host_outputs(pb, trace_len, pso_state, ls_trials)
        b = C.c_size_t()
        _check(lib.zeus_server_request_bytes(C.byref(pb), C.byref(r), C.byref(b)))
        return b.value

    def submit(self, problem, *, trace_len=0, pso_state=False, ls_trials=True) -> int:
        pb = problem if isinstance(problem, zeus_problem) else make_problem(problem)
        o, s, r = _host_outputs(pb, trace_len, pso_state, ls_trials)
        t = C.c_uint64()
        _check(lib.zeus_server_submit(self.h, C.byref(pb), C.byref(r), C.byref(t)))
        self._live[t.value] = (pb, o, s, r)
        return t.value

    def wait(self, ticket: int, timeout_s=None):
        """Results of a ticket (host arrays, summary and times in ns), or None
        when a poll (timeout_s == 0) finds it unfinished."""
        tm = zeus_request_times()
        ns = -1 if timeout_s is None else int(timeout_s * 1e9)
        code = lib.zeus_server_wait(self.h, C.c_uint64(ticket), C.c_int64(ns), C.byref(tm))
        if code == NOT_READY:
            return None
        if code not in (OK, ETIMEOUT):
            self._live.pop(ticket, None)   # the ticket is released: its arrays are no longer written
        _check(code)
        _, o, s, _ = self._live.pop(ticket)
        o["summary"] = _summary_dict(s)
        o["times"] = {k: getattr(tm, k) for k, _ in zeus_request_times._fields_}
        return o

    def cancel(self, ticket: int) -> int:
        code = lib.zeus_server_cancel(self.h, C.c_uint64(ticket))
        if code not in (OK, NOT_READY):
            _check(code)
        return code

    def close(self):
        if self.h:
            _check(lib.zeus_server_destroy(self.h))
            self.h = C.c_void_p()
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class DevicePlan:
    """A batch captured into a HIP graph (zeus_plan_*), with torch-owned device
    workspace and outputs; launch() replays the whole solve."""

    def __init__(self, ctx, problems, device="cuda:0", trace_len=0):
        import torch
        self.pbs = (zeus_problem * len(problems))(
            *[p if isinstance(p, zeus_problem) else make_problem(p) for p in problems])
        n = len(problems)
        wb = C.c_size_t()
        _check(lib.zeus_plan_workspace_bytes(self.pbs, n, C.byref(wb)))
        dev = torch.device(device)
        self.ws = torch.empty(wb.value + 256, dtype=torch.uint8, device=dev)
        ws_ptr = (self.ws.data_ptr() + 255) // 256 * 256
        f64, i32 = torch.float64, torch.int32
        self.t = []
        res = (zeus_result * n)()
        for k in range(n):
            nn, d = self.pbs[k].n_starts, self.pbs[k].dim
            t = {"f": torch.empty(nn, dtype=f64, device=dev),
                 "x": torch.empty((nn, d), dtype=f64, device=dev),
                 "iters": torch.empty(nn, dtype=i32, device=dev),
                 "status": torch.empty(nn, dtype=i32, device=dev),
                 "ls_trials": torch.empty(nn, dtype=i32, device=dev),
                 "skips": torch.empty(nn, dtype=i32, device=dev),
                 "resets": torch.empty(nn, dtype=i32, device=dev),
                 "summary": torch.empty(C.sizeof(zeus_summary), dtype=torch.uint8, device=dev)}
            if trace_len:
                t["trace"] = torch.empty((nn, trace_len, d), dtype=f64, device=dev)
            self.t.append(t)
            pp = lambda key: t[key].data_ptr() if key in t else None
            res[k] = zeus_result(f=pp("f"), x=pp("x"), iters=pp("iters"), status=pp("status"),
                                 ls_trials=pp("ls_trials"), trace=pp("trace"),
                                 trace_len=int(trace_len), reserved0=0, summary=pp("summary"),
                                 skips=pp("skips"), resets=pp("resets"))
        self.res = res
        self.h = C.c_void_p()
        _check(lib.zeus_plan_create(ctx, self.pbs, n, C.c_void_p(ws_ptr), wb, self.res,
                                    C.byref(self.h)))

    def launch(self, stream_ptr: int = 0):
        _check(lib.zeus_plan_launch(self.h, C.c_void_p(stream_ptr) if stream_ptr else None))

    def host(self) -> list:
        out = []
        for t in self.t:
            o = {k: v.cpu().numpy() for k, v in t.items() if k != "summary"}
            s = zeus_summary.from_buffer_copy(bytes(t["summary"].cpu().numpy().tobytes()))
            o["summary"] = _summary_dict(s)
            out.append(o)
        return out

    def close(self):
        if self.h:
            _check(lib.zeus_plan_destroy(self.h))
            self.h = C.c_void_p()


class DeviceSolve:
    """Device-resident buffers (torch tensors) for zeus_minimize_async."""

    def __init__(self, problem: dict, device="cuda:0", trace_len=0, pso_state=False):
        import torch
        self.pb = make_problem(problem)
        n, d = self.pb.n_starts, self.pb.dim
        dev = torch.device(device)
        ws = zeus_workspace_bytes(self.pb)
        self.ws = torch.empty(ws + 256, dtype=torch.uint8, device=dev)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.ws_bytes = ws
        f64, i32 = torch.float64, torch.int32
        self.t = {"f": torch.empty(n, dtype=f64, device=dev),
                  "x": torch.empty((n, d), dtype=f64, device=dev),
                  "iters": torch.empty(n, dtype=i32, device=dev),
                  "status": torch.empty(n, dtype=i32, device=dev),
                  "ls_trials": torch.empty(n, dtype=i32, device=dev),
                  "skips": torch.empty(n, dtype=i32, device=dev),
                  "resets": torch.empty(n, dtype=i32, device=dev),
                  "summary": torch.empty(C.sizeof(zeus_summary), dtype=torch.uint8, device=dev)}
        if pso_state:
            self.t.update(seeds=torch.empty((n, d), dtype=f64, device=dev),
                          pso_v=torch.empty((n, d), dtype=f64, device=dev),
                          pso_px=torch.empty((n, d), dtype=f64, device=dev),
                          pso_pf=torch.empty(n, dtype=f64, device=dev),
                          pso_best_x=torch.empty(d, dtype=f64, device=dev))
        if trace_len:
            self.t["trace"] = torch.empty((n, trace_len, d), dtype=f64, device=dev)
        p = lambda k: self.t[k].data_ptr() if k in self.t else None
        self.result = zeus_result(f=p("f"), x=p("x"), iters=p("iters"), status=p("status"),
                                  ls_trials=p("ls_trials"), seeds=p("seeds"), pso_v=p("pso_v"),
                                  pso_px=p("pso_px"), pso_pf=p("pso_pf"),
                                  pso_best_x=p("pso_best_x"), trace=p("trace"),
                                  trace_len=int(trace_len), reserved0=0, summary=p("summary"),
                                  skips=p("skips"), resets=p("resets"))

    def enqueue(self, ctx, stream_ptr: int = 0):
        zeus_minimize_async(ctx, self.pb, self.ws_ptr, self.ws_bytes, self.result, stream_ptr)

    def enqueue_static(self, ctx, stream_ptr: int = 0):
        """The same solve in the library's fixed workspace (this object's own
        workspace tensor is not used)."""
        zeus_minimize_async_static(ctx, self.pb, self.result, stream_ptr)

    def summary(self) -> dict:
        raw = bytes(self.t["summary"].cpu().numpy().tobytes())
        s = zeus_summary.from_buffer_copy(raw)
        return {k: getattr(s, k) for k, _ in zeus_summary._fields_}

    def host(self) -> dict:
        out = {k: v.cpu().numpy() for k, v in self.t.items() if k != "summary"}
        out["summary"] = self.summary()
        return out
