"""Pair coefficients of the collision kinematics and kernel (oracle; test infrastructure).

Sources in the paper:
* post-collision velocities in relative-velocity form (Sec. 4, first display):
  v' = v - a g + a|g| sigma,  v'_* = v - a g - b|g| sigma  with
  a = m_j/(m_i+m_j), b = m_i/(m_i+m_j);
* the dimensionless VSS/VHS kernel (Sec. 3, eq. NVSS) and the Knudsen number
  Kn_ij (Sec. 3, eq. Kn);
* the support ball S and the anti-aliasing condition (Sec. 4, eq. domain), R = 2S.
"""
from __future__ import annotations

import math

K_B = 1.380649e-23  # Boltzmann constant, J/K


def pair_ab(mi: float, mj: float) -> tuple[float, float]:
    """(a, b) = (m_j/(m_i+m_j), m_i/(m_i+m_j))."""
    return mj / (mi + mj), mi / (mi + mj)


def gamma_exponent(omega: float) -> float:
    """Power of |g| in the VSS kernel: 2(1 - omega) (Sec. 2, eq. VSS)."""
    return 2.0 * (1.0 - omega)


def vss_prefactor(mi: float, mj: float, omega: float, alpha: float = 1.0, kn0: float = 1.0) -> float:
    """C_ij = Kn_ij^{-1} times the constant of the dimensionless kernel (eq. NVSS).

    Kn_ij^{-1} carries sqrt(1 + m_i/m_j) (eq. Kn) and the kernel constant divides by
    it, so the product is alpha / (Kn0 2^{1+alpha} Gamma(2.5-omega) pi mu_ij^{omega-1/2})
    with mu_ij = m_i m_j/(m_i+m_j) and Kn0 = 1/(pi n0 d_ref^2 (T_ref/T0)^{omega-1/2} H0).
    It is symmetric in (i, j), as the weak forms of Sec. 2 require.
    """
    mu = mi * mj / (mi + mj)
    return alpha / (kn0 * 2.0 ** (1.0 + alpha) * math.gamma(2.5 - omega) * math.pi * mu ** (omega - 0.5))


def knudsen(mi: float, mj: float, n0: float, d_ref: float, T_ref: float, T0: float,
            omega: float, H0: float) -> float:
    """Kn_ij of Sec. 3 (eq. Kn), SI inputs."""
    return 1.0 / (math.sqrt(1.0 + mi / mj) * math.pi * n0 * d_ref ** 2 * (T_ref / T0) ** (omega - 0.5) * H0)


def reference_speed(T0: float, m0: float) -> float:
    """u0 = sqrt(2 k_B T0 / m0) (Sec. 3)."""
    return math.sqrt(2.0 * K_B * T0 / m0)


def support_radius(L: float, mi: float, mj: float) -> float:
    """Largest S allowed by the anti-aliasing condition (Sec. 4, eq. domain) for the
    ordered pair (i, j): 2L = (max(4 m_j/(m_i+m_j), 2) + sqrt(1 + m_j/m_i)) S + S."""
    return 2.0 * L / (max(4.0 * mj / (mi + mj), 2.0) + math.sqrt(1.0 + mj / mi) + 1.0)


def truncation_radius(L: float, mi: float, mj: float) -> float:
    """R_ij = 2S (Sec. 4, truncation item 2), with S taken as the smaller of the two
    orderings so that the truncated kernel is the same for (i, j) and (j, i)."""
    return 2.0 * min(support_radius(L, mi, mj), support_radius(L, mj, mi))
