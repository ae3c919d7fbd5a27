"""Build the CPU oracle shared library (test infrastructure only).

    python oracle/build.py

Compiles zeus_oracle.c with gcc twice: oracle/libzeus_oracle.so (the
default build, whose rounding order is fixed by the readings in the source)
and oracle/libzeus_oracle_plain.so (-DZO_PLAIN: sums left to right, unfused
row products and update, the C library's sin/cos/exp/log).  No contraction of
multiply-adds (-ffp-contract=off), no fast-math; OpenMP over starts.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libzeus_oracle.so")
LIB_PLAIN = os.path.join(HERE, "libzeus_oracle_plain.so")
FLAGS = ["-O2", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
         "-shared", "-Wall", "-Wextra"]


def _one(out, extra, verbose, flags=FLAGS):
    src = os.path.join(HERE, "zeus_oracle.c")
    tmp = out + ".tmp"
    cmd = ["gcc", *flags, *extra, "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    _one(LIB_PLAIN, ["-DZO_PLAIN"], verbose)
    return _one(LIB, [], verbose)


SAN_FLAGS = ["-O1", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
             "-shared", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined"]


def build_sanitized(out_dir: str, verbose: bool = False) -> dict:
    """Both builds of the oracle with AddressSanitizer and
    UndefinedBehaviorSanitizer, into out_dir (for CPU runs with the sanitizer
    runtimes preloaded).  Returns {"default": path, "plain": path}."""
    os.makedirs(out_dir, exist_ok=True)
    d = _one(os.path.join(out_dir, "libzeus_oracle.so"), [], verbose, SAN_FLAGS)
    p = _one(os.path.join(out_dir, "libzeus_oracle_plain.so"), ["-DZO_PLAIN"], verbose, SAN_FLAGS)
    return {"default": d, "plain": p}


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
