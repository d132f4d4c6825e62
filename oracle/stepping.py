"""Time stepping of the spatially homogeneous problem df^i/dt = sum_j Q^{ij}(f^i, f^j)
(oracle; test infrastructure).

Sec. 5 advances the DG system in time with the second-order strong-stability-preserving
Runge-Kutta scheme, and Sec. 6.1 evolves the Krook-Wu solution with it (time step 0.01).
In the two-stage form of that scheme:

    f1      = f^n + dt L(f^n)
    f^{n+1} = 1/2 f^n + 1/2 (f1 + dt L(f1))

The forward-Euler step f^{n+1} = f^n + dt L(f^n) is its first stage.  Here L is the
collision operator of ``spectral`` (optionally followed by the conservation projection
of ``moments``), or any callable for the scheme's own checks.
"""
from __future__ import annotations

import numpy as np

from . import grids as G
from . import moments as M
from . import spectral as S


def euler(f: np.ndarray, rhs, dt: float, steps: int) -> np.ndarray:
    for _ in range(steps):
        f = f + dt * rhs(f)
    return f


def ssprk2(f: np.ndarray, rhs, dt: float, steps: int) -> np.ndarray:
    for _ in range(steps):
        f1 = f + dt * rhs(f)
        f = 0.5 * f + 0.5 * (f1 + dt * rhs(f1))
    return f


def collision_rhs(prob, Ls=None, project: bool = True):
    """f [s][N][N][N] -> sum_j Q^{ij}, with species grids Ls if given, projected onto the
    collision invariants (FP64 least squares) when project is true."""
    Ls = tuple(Ls) if Ls is not None else (prob.L,) * prob.s

    def rhs(f):
        Q = S.collide(f, prob) if len(set(Ls)) == 1 else G.collide(f, prob, Ls)
        return M.conserve(Q, prob.masses, Ls) if project else Q
    return rhs
