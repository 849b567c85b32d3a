"""Seeded synthetic books shaped like the paper's batched-rebalancing workloads.

This package only draws random numbers and lays data out. It holds none of the
solver's arithmetic and is shared by the oracle tests, the GPU tests, the
smoke entry point and the benchmark.
"""
from .books import (  # noqa: F401
    Universe,
    Book,
    make_config,
    CONFIG_NAMES,
    subset_accounts,
    to_f32_exact,
)
