"""Seeded synthetic problem generators shared by the oracle tests, the GPU
tests and the benchmark.

This package builds operators, initial states, targets and control arrays;
it performs none of the propagation, cost or gradient arithmetic of the
method.  Every function is deterministic in its seed.
"""
from .cqed import (  # noqa: F401
    Workload,
    destroy,
    coherent_ket,
    resonator_problem,
    transmon_resonator_problem,
    dense_random_problem,
    banded_random_problem,
    controls_uniform,
    controls_smooth_noise,
    config_c1,
    config_c2,
    config_c3,
    config_c4,
    serving_requests,
    serving_model,
    serving_controls,
    SERVING_SHAPES,
)
