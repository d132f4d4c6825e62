"""Pins of the kernel mode F and the loss weight G- (Sec. 4) against independent
quadratures and closed forms."""
import numpy as np
import pytest
import scipy.integrate

from oracle import spectral as S


def _sphere_rule(n):
    """Tensor Gauss-Legendre (cos theta) x trapezoid (azimuth), written here
    independently of the oracle's quadrature module."""
    x, w = np.polynomial.legendre.leggauss(n)
    ph = np.arange(2 * n) * np.pi / n
    st = np.sqrt(1 - x * x)
    P = np.stack([np.outer(st, np.cos(ph)).ravel(), np.outer(st, np.sin(ph)).ravel(), np.repeat(x, 2 * n)], 1)
    return P, np.repeat(w, 2 * n) * np.pi / n


@pytest.mark.parametrize("gamma", [0.0, 0.52, 1.0])
def test_F_closed_form_vs_sphere_integral(gamma):
    """F(k, rho) = rho^2 int_{S^2} C rho^gamma e^{-i pi rho a k.g/L} dg (Sec. 4, alpha = 1)."""
    C, L, a = 0.37, 6.0, 2.0 / 3.0
    P, W = _sphere_rule(60)
    rng = np.random.default_rng(1)
    for _ in range(6):
        k = rng.integers(-16, 16, size=3)
        rho = rng.uniform(0.0, 5.4)
        num = rho ** 2 * np.sum(W * C * rho ** gamma * np.exp(-1j * np.pi * rho * a * (P @ k) / L))
        closed = S.kernel_mode_F(np.linalg.norm(k), rho, a, gamma, C, L)
        assert abs(num.imag) < 1e-12
        assert num.real == pytest.approx(closed, rel=1e-11, abs=1e-12)


def test_G_minus_closed_form_maxwell():
    """gamma = 0: int_0^R rho^2 sinc(kappa rho) = (sin kR - kR cos kR)/k^3, R^3/3 at k = 0."""
    R, L, C = 4.53, 5.0, 0.8
    m = np.array([0.0, 1.0, np.sqrt(2.0), 3.0, np.sqrt(75.0), 13.0])
    kap = np.pi * m / L
    with np.errstate(divide="ignore", invalid="ignore"):
        I = np.where(kap > 0, (np.sin(kap * R) - kap * R * np.cos(kap * R)) / kap ** 3, R ** 3 / 3)
    assert np.allclose(S.loss_weight(m, R, 0.0, C, L), 16 * np.pi ** 2 * C * I, rtol=1e-13, atol=1e-13)


def test_G_minus_closed_form_hard_sphere():
    """gamma = 1: int_0^R rho^3 sinc(kappa rho) = (1/k)[-R^2 cos kR/k + 2R sin kR/k^2 + 2(cos kR - 1)/k^3]."""
    R, L, C = 5.437, 6.0, 1.3
    m = np.array([0.0, 1.0, 2.0, np.sqrt(11.0), 9.0, np.sqrt(768.0)])
    k = np.pi * m / L
    with np.errstate(divide="ignore", invalid="ignore"):
        I = np.where(k > 0, (-R * R * np.cos(k * R) / k + 2 * R * np.sin(k * R) / k ** 2
                             + 2 * (np.cos(k * R) - 1) / k ** 3) / k, R ** 4 / 4)
    assert np.allclose(S.loss_weight(m, R, 1.0, C, L), 16 * np.pi ** 2 * C * I, rtol=1e-12, atol=1e-12)


def test_G_minus_fractional_gamma_vs_adaptive():
    """gamma = 0.52 (omega = 0.74): against scipy's adaptive quadrature."""
    R, L, C, gamma = 5.437, 6.0, 1.0, 0.52
    for m in (0.0, 1.0, 5.0, 17.3):
        ref, err = scipy.integrate.quad(lambda r: r ** (gamma + 2) * np.sinc(r * m / L), 0.0, R,
                                        epsabs=1e-14, epsrel=1e-14, limit=400)
        assert S.loss_weight(np.array([m]), R, gamma, C, L)[0] == pytest.approx(16 * np.pi ** 2 * C * ref, rel=1e-12)


def test_G_minus_equals_exact_sphere_gain_at_k0():
    """Mass balance of the continuous weights: G+(l, -l) with the exact sphere integral
    and an exact radial integral equals G-(-l).  Checked with a high-order radial rule."""
    R, L, C, gamma, a = 4.45, 6.0, 0.9, 0.52, 0.4
    rho, w = np.polynomial.legendre.leggauss(400)
    rho, w = 0.5 * R * (rho + 1), 0.5 * R * w
    for labs in (0.0, 1.0, 3.0, 7.5):
        gp = np.sum(w * S.kernel_mode_F(0.0, rho, a, gamma, C, L) * 4 * np.pi * S.sinc(np.pi * rho * labs / L))
        assert gp == pytest.approx(S.loss_weight(np.array([labs]), R, gamma, C, L)[0], rel=1e-6)
