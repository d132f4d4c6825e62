"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and the bench.

This package only samples distribution functions on the velocity grid and draws
random parameters; it holds none of the collision operator's arithmetic.
"""
from .inputs import (  # noqa: F401
    velocity_grid,
    maxwellian,
    config,
    CONFIGS,
    draw_bimaxwellian_batch,
    draw_config3_batch,
)
