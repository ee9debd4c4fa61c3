"""Seeded synthetic workloads for the block-Toeplitz array operator.

This package produces inputs only: generator blocks Z_{m,n}, rim coupling
blocks and right-hand sides.  It holds none of the apply/solve arithmetic, so
both the CPU oracle and the GPU library can consume it without sharing any of
the method's code.  See ``synth.arrays`` for the recipe.
"""
from .arrays import (  # noqa: F401
    Problem,
    make_problem,
    make_config,
    rhs_random,
    rhs_plane_wave,
    rhs_ports,
    serving_stream,
    CONFIGS,
    SEED_BASE,
)
