"""CPU oracle of the batched multistart method (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.
"""
