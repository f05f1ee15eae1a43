"""Seeded synthetic inputs shared by the FP64 oracle and the GPU harness.

This package only builds inputs: tetrahedral grid meshes, pinned vertex sets,
initial states and material parameters. It contains none of the solver's
arithmetic (no deformation gradients, masses, stiffness fits, energies or
solves), so that the oracle and the HIP path stay independent of each other.
"""
from .grid import (  # noqa: F401
    GRAVITY,
    Material,
    Workload,
    kuhn_grid,
    pinned_face,
    workload_cantilever,
    workload_block,
    workload_mixed_cantilever,
    workload_fiber_cantilever,
    cantilever_ground_planes,
    workload_batch,
    workload_pool,
    spline_knots,
    spline_d2_multipliers,
    lame_from_young,
    make_material,
    NEOHOOKEAN,
    STVK,
    SPLINE,
    COROTATED,
    POLYNOMIAL,
    MOONEY_RIVLIN,
    MATERIAL_NAMES,
)
