"""Quadrature rules of the fast method (oracle; test infrastructure).

Sec. 4: the radial integral over [0, R] uses Gauss-Legendre with N_rho = O(N)
points; the sphere uses an M-point spherical design with equal weights 4 pi / M.

The published design files the paper cites are not available, so the designs are
built from their definitions:
* M = 6:  the octahedron, +-e_x, +-e_y, +-e_z (a spherical 3-design);
* M = 12: the icosahedron, cyclic permutations of (0, +-1, +-phi)/sqrt(1+phi^2)
  (a 5-design);
* M = 24: the orbit of one point under the 24 rotations of the cube.  An orbit of
  the rotation group is a 7-design exactly when the group-invariant harmonics of
  degree <= 7 vanish at the generating point.  Those are the cubic harmonics of
  degree 4 and 6; on the unit sphere they vanish when (x^2, y^2, z^2) are the three
  roots of 105 t^3 - 105 t^2 + 21 t - 1 = 0.  The generating point takes the
  positive square roots in increasing order.  The design is chiral and not
  antipodal.

Point order: points are sorted lexicographically by (x, y, z).
"""
from __future__ import annotations

import itertools

import numpy as np


def gauss_legendre(R: float, n: int) -> tuple[np.ndarray, np.ndarray]:
    """Gauss-Legendre nodes and weights on [0, R]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * R * (x + 1.0), 0.5 * R * w


def _lexsort(P: np.ndarray) -> np.ndarray:
    order = np.lexsort((P[:, 2], P[:, 1], P[:, 0]))
    return P[order]


def cube_rotations() -> list[np.ndarray]:
    """The 24 signed permutation matrices of determinant +1."""
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1.0, -1.0), repeat=3):
            R = np.zeros((3, 3))
            for r in range(3):
                R[r, perm[r]] = signs[r]
            if np.linalg.det(R) > 0:
                out.append(R)
    return out


def spherical_design(M: int) -> np.ndarray:
    """Design points, shape (M, 3), float64."""
    if M == 6:
        P = np.concatenate([np.eye(3), -np.eye(3)])
    elif M == 12:
        phi = (1.0 + np.sqrt(5.0)) / 2.0
        base = []
        for s1 in (1.0, -1.0):
            for s2 in (1.0, -1.0):
                base.append((0.0, s1, s2 * phi))
        pts = []
        for (x, y, z) in base:
            pts += [(x, y, z), (z, x, y), (y, z, x)]
        P = np.array(pts) / np.sqrt(1.0 + phi * phi)
    elif M == 24:
        t = np.sort(np.roots([105.0, -105.0, 21.0, -1.0]).real)
        p = np.sqrt(t)
        P = np.array([R @ p for R in cube_rotations()])
    else:
        raise ValueError(f"no spherical design with M={M}")
    return _lexsort(P)


def design_quadrature(M: int) -> tuple[np.ndarray, np.ndarray]:
    """(points, weights) with equal weights 4 pi / M."""
    P = spherical_design(M)
    return P, np.full(M, 4.0 * np.pi / M)


def product_sphere_rule(n: int) -> tuple[np.ndarray, np.ndarray]:
    """Gauss-Legendre in cos(theta) (n points) times the trapezoid rule in the
    azimuth (2n points); exact for spherical harmonics of degree <= 2n-1.
    Used only to show convergence of the sphere sum as the rule is refined."""
    x, w = np.polynomial.legendre.leggauss(n)
    phis = np.arange(2 * n) * (np.pi / n)
    st = np.sqrt(1.0 - x * x)
    P = np.stack([
        (st[:, None] * np.cos(phis)[None, :]).ravel(),
        (st[:, None] * np.sin(phis)[None, :]).ravel(),
        np.repeat(x, 2 * n),
    ], axis=1)
    W = np.repeat(w, 2 * n) * (np.pi / n)
    return P, W


def is_antipodal(P: np.ndarray, tol: float = 1e-12) -> bool:
    """True when -p is a point of the set for every point p."""
    return all(np.min(np.linalg.norm(P + p, axis=1)) < tol for p in P)
