"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only produces data: radial node sets, initial velocity fields and
ensemble member parameters.  It contains none of the solver's arithmetic (no
finite differences, transforms or linear solves), so both the CPU oracle and the
HIP library can be fed from it without sharing code.
"""
from .synth import (  # noqa: F401
    chebyshev_nodes,
    splitmix64,
    normals,
    uniforms,
    make_state,
    workload_state,
    laminar_state,
    ensemble_members,
    WORKLOADS,
)
