"""Seeded synthetic workloads shared by the oracle tests, the HIP parity tests
and the benchmark.

This package only draws numbers: data sets, initial parameter vectors, masks
and per-chain starting points.  It contains none of the sampler's arithmetic
(no network evaluation, no potential, no gradient, no integrator), so that the
oracle and the HIP path stay independent of each other.
"""

from .synth import (  # noqa: F401
    Workload,
    CONFIG_NAMES,
    make,
    n_params,
    tower_param_count,
)
