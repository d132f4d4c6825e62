"""MI355X (gfx950) multi-species fast Fourier spectral collision operator.

The library (libdgfs.so, C ABI in include/dgfs.h) evaluates
Q^i = sum_j Q^{ij}(f^i, f^j) for a batch of independent spatial points with hand-written
HIP kernels; this package is its thin Python binding.
"""
from .collision import (  # noqa: F401
    CollisionGroup,
    CollisionPlan,
    Slab,
    slab_gll,
    Graph,
    tile_candidates,
    check_problem,
    design,
    interpolation_matrix,
    kernel_mode,
    pair_tables,
    vhs_kernel,
    vss_kernel,
    pair_prefactor,
)
