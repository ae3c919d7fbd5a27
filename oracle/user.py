"""User-defined objectives for the oracle (test infrastructure).

The user's source (the same text the GPU path compiles with hipRTC) is
compiled for the CPU with g++ against user_objective.hpp -- the oracle's own
dual numbers and its sin, cos, exp, log -- into a shared library whose two
entry points are registered with the oracle's zo_set_user.  The oracle then
evaluates objective 7 (ZO_USER) through them: the value in double, and Alg. 5
as written (one dual evaluation per direction).
"""
import ctypes as C
import hashlib
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))

SHIM = r'''
#include "user_objective.hpp"
#include <vector>
#line 1 "objective"
{source}
extern "C" double zo_user_value(const double *x, int d) {{ return objective<double>(x, d); }}
extern "C" double zo_user_dual(const double *xv, const double *xt, int d, double *t) {{
  std::vector<zeus::Dual> x((size_t)d);
  for (int i = 0; i < d; ++i) x[(size_t)i] = zeus::Dual(xv[i], xt[i]);
  const zeus::Dual r = objective<zeus::Dual>(x.data(), d);
  *t = r.t;
  return r.v;
}}
'''

_VALUE = C.CFUNCTYPE(C.c_double, C.POINTER(C.c_double), C.c_int)
_DUAL = C.CFUNCTYPE(C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int,
                    C.POINTER(C.c_double))
_loaded = {}


def build(source: str) -> str:
    """Compiles a user source into a shared library (cached by content)."""
    with open(os.path.join(HERE, "user_objective.hpp")) as f:
        hdr = f.read()
    key = hashlib.sha256((hdr + "\0" + source).encode()).hexdigest()[:16]
    out_dir = os.path.join(tempfile.gettempdir(), "zeus_oracle_user")
    os.makedirs(out_dir, exist_ok=True)
    so = os.path.join(out_dir, f"user_{key}.so")
    if os.path.exists(so):
        return so
    cpp = os.path.join(out_dir, f"user_{key}.cpp")
    with open(cpp, "w") as f:
        f.write(SHIM.format(source=source))
    tmp = so + f".{os.getpid()}.tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-I", HERE, cpp, "-o", tmp, "-L", HERE, "-l:libzeus_oracle.so", f"-Wl,-rpath,{HERE}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"user objective does not compile for the oracle:\n{r.stderr}")
    os.replace(tmp, so)
    return so


def use(source: str, oracle_lib):
    """Registers the user objective with the oracle library (process-wide)."""
    so = build(source)
    if so not in _loaded:
        L = C.CDLL(so)
        _loaded[so] = (L, _VALUE(("zo_user_value", L)), _DUAL(("zo_user_dual", L)))
    _, fv, fd = _loaded[so]
    oracle_lib.zo_set_user.argtypes = [_VALUE, _DUAL]
    oracle_lib.zo_set_user(fv, fd)
    return so
