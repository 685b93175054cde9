"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only builds matrices and right-hand sides (index arithmetic and
random draws); it contains none of the solver's arithmetic.
"""
from .stencils import (  # noqa: F401
    Problem,
    grid_laplacian,
    random_spd,
    random_pattern,
    make_config,
    rhs,
    weighted_grid,
    grid_batch,
    convection_diffusion,
    CONFIG_NAMES,
)
from .elasticity import elasticity3d, element_stiffness, material_matrix, strain_matrix  # noqa: F401
from .update_panels import update_panels  # noqa: F401
