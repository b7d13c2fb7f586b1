"""Seeded synthetic workloads shared by the CPU oracle and the HIP path.

This package only draws numbers (geometries, basis exponents, coefficients,
determinant lists, network parameters, walkers).  It holds none of the
method's arithmetic, so both implementations can consume it without sharing
any computation.
"""

from .configs import (  # noqa: F401
    System,
    NetShape,
    Workload,
    make_config,
    make_system_workload,
    make_serving_jobs,
    param_count,
    CONFIG_NAMES,
)
