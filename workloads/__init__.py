"""Seeded synthetic inputs for the pressure-Poisson solve.

This package holds only input generation: source fields on a Cartesian grid
and target point sets (grid nodes, ellipses, fish-like body surfaces and their
lifted copies).  It contains none of the solve's arithmetic (no Green's
function, no expansions), so both the CPU oracle and the GPU path may use it.
"""

from .generators import (  # noqa: F401
    GridSpec,
    grid_nodes,
    gaussian_source,
    lamb_oseen_params,
    vortex_source,
    band_mask,
    envelope_weight,
    ellipse_targets,
    fish_surface_targets,
    workload,
    WORKLOADS,
)
