"""Zeus batched multistart (PSO -> BFGS with forward-mode dual-number
gradients) for AMD Instinct MI355X (gfx950).

The compute path lives in ``libzeus.so`` (hand-written HIP kernels behind a
C ABI declared in ``include/zeus.h``); ``zeus`` is the thin ctypes binding.
"""
