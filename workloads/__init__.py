"""Seeded synthetic inputs shared by the FP64 oracle and the GPU library.

This package only *constructs inputs* (sparse operators, right-hand sides,
tall-skinny test blocks).  It contains none of the solver's or the block
orthogonalization's arithmetic, and it imports neither the oracle nor the
GPU package.
"""
from .generators import (  # noqa: F401
    CSR,
    laplace2d,
    laplace3d,
    convdiff2d,
    convdiff_params,
    variable_width,
    uniform_vector,
    rhs_from_solution,
    gaussian_block,
    logscaled_block,
    glued_block,
    nearly_dependent_panel,
    ill_conditioned_panel,
    laplace_eigpair_2d,
    laplace_eigpair_3d,
    laplace_extreme_eigs,
    make_problem,
)
