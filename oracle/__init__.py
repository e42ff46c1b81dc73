"""Reference oracle (test infrastructure only).

A plain FP64 CPU implementation of the multi-time-step PD/FE coupling written
from the paper (arXiv 2403.03605); it shares no code with the HIP library.  Only
the tests, the smoke check and the benchmark's CPU-baseline leg may use it.
"""
from .oracle import Oracle, build_oracle, neighbors_brute, neighbors_grid, exp_moment  # noqa: F401
