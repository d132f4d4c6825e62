"""Moments, the Maxwellian and the FP64 conservation projection (oracle; test infrastructure).

* moments of Sec. 3 (nondimensional): n^i = int f^i, u^i = int v f^i / n^i,
  T^i = (2 m_i / (3 n^i)) int |v - u^i|^2 f^i;
* the collision invariants of Sec. 2 (eq. consv): per-species number, total momentum
  sum_i m_i int v Q^i and total energy sum_i m_i int |v|^2 Q^i;
* the conservation projection.  The paper does not correct conservation itself; its
  introduction credits a Lagrangian post-processing to earlier work.  Here it is the
  least-squares projection of Q onto the constraint set A Q = 0:
      Q~ = Q - A^T (A A^T)^{-1} A Q,
  with one row per species number (s rows), three momentum rows and one energy row,
  each integral taken with the rectangle rule (weight h_i^3 on species i's grid).
"""
from __future__ import annotations

import numpy as np


def grid(N: int, L: float) -> np.ndarray:
    return -L + np.arange(N) * (2.0 * L / N)


def moments(f: np.ndarray, m: float, L: float) -> dict:
    """n, u (3), T of one species sampled on the grid of half-width L."""
    N = f.shape[0]
    h3 = (2.0 * L / N) ** 3
    v = grid(N, L)
    VX, VY, VZ = np.meshgrid(v, v, v, indexing="ij")
    n = f.sum() * h3
    u = np.array([(VX * f).sum(), (VY * f).sum(), (VZ * f).sum()]) * h3 / n
    c2 = (VX - u[0]) ** 2 + (VY - u[1]) ** 2 + (VZ - u[2]) ** 2
    T = 2.0 * m / (3.0 * n) * (c2 * f).sum() * h3
    return {"n": n, "u": u, "T": T}


def constraint_matrix(masses, Ls, N: int) -> np.ndarray:
    """Rows (s + 4) x (s N^3): species number, m-weighted momentum (3), energy."""
    s = len(masses)
    A = np.zeros((s + 4, s * N ** 3))
    for i in range(s):
        h3 = (2.0 * Ls[i] / N) ** 3
        v = grid(N, Ls[i])
        VX, VY, VZ = np.meshgrid(v, v, v, indexing="ij")
        sl = slice(i * N ** 3, (i + 1) * N ** 3)
        A[i, sl] = h3
        A[s + 0, sl] = masses[i] * h3 * VX.ravel()
        A[s + 1, sl] = masses[i] * h3 * VY.ravel()
        A[s + 2, sl] = masses[i] * h3 * VZ.ravel()
        A[s + 3, sl] = masses[i] * h3 * (VX ** 2 + VY ** 2 + VZ ** 2).ravel()
    return A


def invariants(Q: np.ndarray, masses, Ls) -> np.ndarray:
    """A Q for Q shaped [s][N][N][N]."""
    s, N = Q.shape[0], Q.shape[1]
    return constraint_matrix(masses, Ls, N) @ Q.reshape(-1)


def conservation_residual(Q: np.ndarray, masses, Ls) -> np.ndarray:
    """|A Q| / (|A| |Q|) per constraint row (elementwise absolute values)."""
    s, N = Q.shape[0], Q.shape[1]
    A = constraint_matrix(masses, Ls, N)
    q = Q.reshape(-1)
    return np.abs(A @ q) / (np.abs(A) @ np.abs(q))


def conserve(Q: np.ndarray, masses, Ls) -> np.ndarray:
    """Least-squares projection onto the conserving set, FP64."""
    s, N = Q.shape[0], Q.shape[1]
    A = constraint_matrix(masses, Ls, N)
    q = Q.reshape(-1).astype(np.float64)
    lam = np.linalg.solve(A @ A.T, A @ q)
    return (q - A.T @ lam).reshape(Q.shape)
