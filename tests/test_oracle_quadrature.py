"""Pins of the oracle's quadrature rules against their defining exactness properties."""
import numpy as np
import pytest
from scipy.special import eval_legendre

from oracle import quadrature as Qd


def _harmonic_energy(P, n):
    """sum_{p,p'} P_n(sigma_p . sigma_p') = (4 pi/(2n+1)) sum_m |sum_p Y_nm(sigma_p)|^2 >= 0."""
    G = np.clip(P @ P.T, -1.0, 1.0)
    return float(np.sum(eval_legendre(n, G)))


@pytest.mark.parametrize("M,t", [(6, 3), (12, 5), (24, 7)])
def test_design_strength(M, t):
    P, W = Qd.design_quadrature(M)
    assert P.shape == (M, 3)
    assert np.allclose(np.linalg.norm(P, axis=1), 1.0, atol=1e-15)
    assert W.sum() == pytest.approx(4 * np.pi, rel=1e-15)
    for n in range(1, t + 1):
        assert abs(_harmonic_energy(P, n)) < 1e-12 * M * M, (M, n)
    assert _harmonic_energy(P, t + 1) > 1e-3, (M, t + 1)


def test_design_symmetry():
    assert Qd.is_antipodal(Qd.spherical_design(6))
    assert Qd.is_antipodal(Qd.spherical_design(12))
    assert not Qd.is_antipodal(Qd.spherical_design(24))
    # the 24-point design is one orbit of the cube rotations
    P = Qd.spherical_design(24)
    for R in Qd.cube_rotations():
        Q = P @ R.T
        assert all(np.min(np.linalg.norm(P - q, axis=1)) < 1e-14 for q in Q)


def test_design_integrates_polynomials():
    """Direct check on monomials: the 7-design integrates x^a y^b z^c, a+b+c <= 7,
    exactly (int over S^2 of x^2 = 4 pi/3, x^4 = 4 pi/5, x^2 y^2 = 4 pi/15, x^6 = 4 pi/7)."""
    P, W = Qd.design_quadrature(24)
    x, y, z = P.T
    cases = {(2, 0, 0): 4 * np.pi / 3, (4, 0, 0): 4 * np.pi / 5, (2, 2, 0): 4 * np.pi / 15,
             (6, 0, 0): 4 * np.pi / 7, (2, 2, 2): 4 * np.pi / 105, (1, 0, 0): 0.0, (3, 3, 1): 0.0,
             (4, 2, 0): 4 * np.pi / 35}
    for (a, b, c), exact in cases.items():
        assert W @ (x ** a * y ** b * z ** c) == pytest.approx(exact, abs=1e-14)


@pytest.mark.parametrize("n", [3, 8, 16])
def test_gauss_legendre_exact_degree(n):
    R = 4.3
    rho, w = Qd.gauss_legendre(R, n)
    assert np.all((rho > 0) & (rho < R))
    for d in range(0, 2 * n):
        assert w @ rho ** d == pytest.approx(R ** (d + 1) / (d + 1), rel=1e-13)
    if n <= 8:   # beyond that the error of degree 2n falls below round-off
        assert abs(w @ rho ** (2 * n) - R ** (2 * n + 1) / (2 * n + 1)) > 1e-12 * R ** (2 * n + 1)


def test_product_sphere_rule_exactness():
    P, W = Qd.product_sphere_rule(5)
    for n in range(1, 10):
        assert abs(W @ eval_legendre(n, P @ np.array([0.3, -0.5, 0.81]) / np.linalg.norm([0.3, -0.5, 0.81]))) < 1e-13
