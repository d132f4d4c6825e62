"""Plain CPU FP64 oracle for the multi-species fast Fourier spectral collision operator.

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU-baseline leg
of the benchmark import this package; the product library never does.  It shares
no code with the HIP path: the only common module is ``synth`` (seeded inputs).

Contents, each following the paper (Jaiswal, Alexeenko & Hu, "A discontinuous
Galerkin fast spectral method for the multi-species Boltzmann equation"):

* ``params``      pair coefficients, VHS/VSS prefactor, Knudsen numbers, the
                  truncation radius from the anti-aliasing condition (Secs. 2-4).
* ``quadrature``  Gauss-Legendre radial rule, spherical designs (Sec. 4).
* ``spectral``    Fourier coefficients, kernel mode F, loss weight G^-, the direct
                  O(N^6) spectral sum, the fast sum, and the exact-sphere variant.
* ``vss``         the sigma-dependent kernel mode of the VSS kernels, alpha in (1, 2]
                  (Sec. 2 eq. VSS, Sec. 4 below eq. GG).
* ``moments``     moments, the Maxwellian, the FP64 conservation projection.
* ``bkw``         the Krook-Wu exact solution and its time derivative (Sec. 6.1).
* ``grids``       species-specific velocity grids: trigonometric interpolation between
                  grids and the pairwise evaluation on the wider grid (the remedy the
                  remark after eq. (domain) in Sec. 4 names and leaves for later).
* ``stepping``    forward Euler and the second-order SSP Runge-Kutta scheme of Sec. 5
                  for the spatially homogeneous problem.
* ``dg``          the nodal DG discretisation of a 1-D slab (Sec. 5): GLL points, upwind
                  flux, diagonal mass and collision tensor, inflow and diffuse-wall
                  boundaries (Sec. 2).
"""
from . import params, quadrature, vss, spectral, moments, bkw, grids, stepping, dg  # noqa: F401
