"""The Krook-Wu exact solution for a binary mixture (Sec. 6.1; oracle, test infrastructure).

Constant kernel B_ij = B_ji = lambda_ji / (4 pi n^(j)) (so omega = 1, alpha = 1 and
the pair prefactor is that constant).  The paper's choice: n1 = n2 = 1,
lambda_11 = lambda_22 = 1, lambda_12 = lambda_21 = 1/2.

f^i(t, v) = n^i (m_i/(2 pi K))^{3/2} exp(-m_i v^2/(2K)) ((1 - 3 Q_i) + (m_i/K) Q_i v^2)

with mu, p_i, A, B, Q(t), Q_i = p_i Q, K(t) and the time derivatives as printed in
Sec. 6.1.
"""
from __future__ import annotations

import numpy as np


class KrookWu:
    def __init__(self, m1: float, m2: float, n1: float = 1.0, n2: float = 1.0,
                 lam11: float = 1.0, lam22: float = 1.0, lam12: float = 0.5, lam21: float = 0.5):
        self.m = (m1, m2)
        self.n = (n1, n2)
        self.lam = {(1, 1): lam11, (2, 2): lam22, (1, 2): lam12, (2, 1): lam21}
        mu = 4.0 * m1 * m2 / (m1 + m2) ** 2
        self.mu = mu
        self.p1 = lam22 - lam21 * mu * (3.0 - 2.0 * mu)
        self.p2 = lam11 - lam12 * mu * (3.0 - 2.0 * mu)
        self.A = (lam11 + lam21 * mu * (3.0 - 2.0 * mu * self.p2 / self.p1)) / 6.0
        self.B = (lam11 * self.p1 + lam21 * mu * (3.0 - 2.0 * mu) * self.p2) / 3.0
        # the solvability condition of Sec. 6.1
        self.condition = (self.p1 - self.p2) * (2.0 * mu ** 2 * (lam21 / self.p1 - lam12 / self.p2) - 1.0)

    def kernel_constant(self, i: int, j: int) -> float:
        """B_ij = lambda_ji / (4 pi n^(j)), species numbered 1, 2."""
        return self.lam[(j, i)] / (4.0 * np.pi * self.n[j - 1])

    def Q(self, t):
        return self.A / (self.A * np.exp(self.A * t) - self.B)

    def dQ(self, t):
        e = np.exp(self.A * t)
        return -self.A ** 3 * e / (self.A * e - self.B) ** 2

    def K(self, t):
        n1, n2 = self.n
        S = n1 + n2
        return S / (S + 2.0 * (n1 * self.p1 + n2 * self.p2) * self.Q(t))

    def dK(self, t):
        n1, n2 = self.n
        S = n1 + n2
        P = n1 * self.p1 + n2 * self.p2
        return -2.0 * S * P / (S + 2.0 * P * self.Q(t)) ** 2 * self.dQ(t)

    def p(self, i: int) -> float:
        return self.p1 if i == 1 else self.p2

    def f(self, i: int, t: float, v2):
        m = self.m[i - 1]
        K = self.K(t)
        Qi = self.p(i) * self.Q(t)
        g = self.n[i - 1] * (m / (2.0 * np.pi * K)) ** 1.5 * np.exp(-m * v2 / (2.0 * K))
        return g * ((1.0 - 3.0 * Qi) + (m / K) * Qi * v2)

    def dfdt(self, i: int, t: float, v2):
        m = self.m[i - 1]
        K, dK = self.K(t), self.dK(t)
        Qi, dQi = self.p(i) * self.Q(t), self.p(i) * self.dQ(t)
        fi = self.f(i, t, v2)
        g = self.n[i - 1] * (m / (2.0 * np.pi * K)) ** 1.5 * np.exp(-m * v2 / (2.0 * K))
        return (fi * (-1.5 * dK / K + m * v2 * dK / (2.0 * K ** 2))
                + g * (-3.0 * dQi + (m / K) * dQi * v2 - (m / K ** 2) * dK * Qi * v2))

    def on_grid(self, N: int, L: float, t: float):
        """(f [2][N^3], df/dt [2][N^3]) on the grid v_n = -L + n 2L/N."""
        v = -L + np.arange(N) * (2.0 * L / N)
        V2 = v[:, None, None] ** 2 + v[None, :, None] ** 2 + v[None, None, :] ** 2
        f = np.stack([self.f(1, t, V2), self.f(2, t, V2)])
        df = np.stack([self.dfdt(1, t, V2), self.dfdt(2, t, V2)])
        return f, df
