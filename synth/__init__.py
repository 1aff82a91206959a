"""Seeded synthetic inputs shared by the tests, the bench and the CPU oracle.

This package only draws random structures and values. It holds none of the
SpMV, conversion, feature or network arithmetic; both the HIP library and the
oracle receive what it produces as plain arrays.
"""
from .matrices import (  # noqa: F401
    Matrix,
    laplacian2d,
    banded,
    poisson_random,
    block_diagonal,
    stencil3d,
    power_law,
    shuffled,
    config1_matrix,
    config2_spec,
    config2_matrix,
    config3_matrix,
    config4_specs,
    config4_matrix,
    config5_specs,
    config5_matrix,
    uniform_vector,
    random_rect,
    from_coords,
    CFG5_FAMILIES,
    CFG5X_FAMILIES,
    CFG5X_TRAIN,
    CFG5X_HELDOUT,
)
from .mlp_inputs import glorot_params, epoch_permutations  # noqa: F401
