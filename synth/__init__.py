"""Seeded synthetic workloads for ptychographic forward/adjoint tests and benchmarks.

This package only draws inputs (objects, probes, scan positions, noise). It holds
none of the forward model's arithmetic: no propagation, no patch extraction, no
loss. Both the FP64 oracle and the GPU path consume what it returns.
"""
from .workloads import (  # noqa: F401
    Problem,
    make_config,
    make_batched_config,
    perturb,
    poisson_counts,
    smooth_field,
)
