"""Seeded synthetic inputs for the space-time heat-equation workloads.

This package only *draws* problem data (coefficient fields, sources, initial
data) with numpy's PCG64 generator.  It contains none of the solver's
arithmetic: no spatial operator, no time stepping, no transform.  Both the CPU
oracle and the GPU library consume what it produces, and neither imports the
other.
"""
from .workloads import (  # noqa: F401
    Problem,
    heat1d_random,
    heat2d_gaussians,
    heat3d_lognormal,
    heat3d_sine,
    heat2d_sine,
    batch2d,
    lognormal_field,
    manufactured_u,
    small_problem,
    batch2d_problem,
    batch2d_parts,
    heat2d_parts,
    gaussian_factors,
    source_from_factors,
    CONFIG_BUILDERS,
    graded_steps,
)
