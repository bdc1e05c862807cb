"""Seeded synthetic inputs: sparse matrices, nonoverlapping partitions and
right-hand sides.

This package holds no arithmetic of the preconditioner. It only builds the
problem that the method is given (a sparse matrix A, a partition of the
unknowns into N sets, and b), so both the CPU oracle and the GPU library can
be fed the same inputs. Seeds come from NumPy's PCG64 (default_rng).
"""

from .problems import (  # noqa: F401
    CONFIGS,
    Problem,
    box_partition_2d,
    box_partition_3d,
    convdiff_2d,
    elasticity_q1_3d,
    elasticity_training_instances,
    fv_diffusion_2d,
    fv_diffusion_3d,
    high_contrast_kappa_2d,
    layered_elasticity,
    lognormal_kappa_3d,
    make_config,
    one_way_convection_2d,
    poisson_2d,
    rcb_partition,
    rhs,
    stokes_cavity_2d,
    weak_scaling_poisson_3d,
    worked_example_7x7,
)
