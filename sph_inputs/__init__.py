"""Seeded synthetic particle layouts for the WCSPH dam-break workloads.

This package only builds inputs: particle positions, velocities, densities,
the physical constants of each case and the domain box.  It performs none of
the per-step SPH arithmetic (no kernel, no pair terms, no integrator), so the
FP64 oracle and the HIP path can both consume its arrays without sharing any
of the method's code.
"""

from .dambreak import (  # noqa: F401
    CASES,
    CLUSTER_SEED,
    SEED_BASE,
    VEL_SEED_64K,
    Case,
    Layout,
    Physics,
    blob,
    cell_grid,
    column,
    dam_break,
    named_case,
    physics,
    refine,
)
