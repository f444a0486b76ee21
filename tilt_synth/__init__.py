"""Seeded synthetic inputs for the TILT solver and its oracle.

This package holds only input generation: low-rank textures, their warped
and corrupted images, windows and ground-truth transforms.  It contains none
of the solver's arithmetic (no warping for the solve, no Jacobian, no
proximal maps), so both the HIP path and the CPU oracle can read the same
arrays without sharing any solver code.
"""

from .textures import (  # noqa: F401
    Patch,
    make_patch,
    make_batch,
    make_config,
    config_names,
    MASTER_SEED,
    patch_rng,
    inner_problem,
    checkerboard_patch,
    convergence_grid,
    RaslSet,
    rasl_set,
)
