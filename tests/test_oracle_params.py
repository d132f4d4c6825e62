"""Pins of the oracle's parameter formulas against numbers printed in the paper."""
import json
import math
import os

import pytest

from oracle import params as P
from oracle import bkw

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


def test_knudsen_matches_printed_F01():
    """eq. (Kn) reproduces the printed Kn of case F-01 to the printed digits."""
    g = _load("knudsen_F01.json")
    m = {"1": g["m1_kg"], "2": g["m2_kg"]}
    for ij, printed in g["printed_Kn"].items():
        i, j = ij[0], ij[1]
        kn = P.knudsen(m[i], m[j], g["n0_per_m3"], g["d_ref_m"][ij], g["T_ref_K"], g["T0_K"],
                       g["omega"][ij], g["H0_m"])
        assert round(kn, 3) == pytest.approx(printed, abs=1e-12), (ij, kn, printed)


def test_reference_speed_matches_printed():
    g = _load("reference_speeds.json")
    for c in g["cases"]:
        assert round(P.reference_speed(c["T0_K"], c["m0_kg"]), 1) == pytest.approx(c["u0_printed"], abs=1e-9)


def test_prefactor_is_kn_inverse_times_kernel_constant():
    """C_ij from the folded formula equals Kn_ij^{-1} times the constant of eq. (NVSS)
    written out from its two factors, for arbitrary SI parameters."""
    mi, mj = 1.3, 2.9          # nondimensional masses
    omega, alpha = 0.74, 1.36
    n0, d, Tr, T0, H0 = 2.0e21, 4.0e-10, 273.0, 300.0, 1e-3
    kn = P.knudsen(mi, mj, n0, d, Tr, T0, omega, H0)
    mu = mi * mj / (mi + mj)
    kernel_const = alpha / (math.sqrt(1 + mi / mj) * mu ** (omega - 0.5) * 2 ** (1 + alpha)
                            * math.gamma(2.5 - omega) * math.pi)
    kn0 = 1.0 / (math.pi * n0 * d * d * (Tr / T0) ** (omega - 0.5) * H0)
    assert P.vss_prefactor(mi, mj, omega, alpha, kn0) == pytest.approx(kernel_const / kn, rel=1e-14)
    # symmetric in (i, j), as the weak forms require
    assert P.vss_prefactor(mi, mj, omega, alpha) == pytest.approx(P.vss_prefactor(mj, mi, omega, alpha), rel=1e-15)


def test_truncation_radius_satisfies_domain_condition():
    """R = 2S with equality in eq. (domain) for the tighter ordering."""
    for L, mi, mj in [(5.0, 1.0, 2.0), (6.0, 1.0, 4.0), (6.0, 1.0, 20.0), (12.0, 1.0, 1.0)]:
        R = P.truncation_radius(L, mi, mj)
        S = R / 2
        for (a, b) in [(mi, mj), (mj, mi)]:
            need = (max(4 * b / (a + b), 2) + math.sqrt(1 + b / a)) * S + S
            assert need <= 2 * L * (1 + 1e-15)
        # equality for at least one ordering
        gaps = [2 * L - ((max(4 * b / (a + b), 2) + math.sqrt(1 + b / a)) * S + S) for (a, b) in [(mi, mj), (mj, mi)]]
        assert min(abs(x) for x in gaps) < 1e-12
    # self pair: R = 4L/(3+sqrt 2)
    assert P.truncation_radius(5.0, 1.0, 1.0) == pytest.approx(20.0 / (3 + math.sqrt(2)), rel=1e-15)


def test_pair_coefficients_conserve_momentum_and_energy():
    """v' and v'_* in relative-velocity form (Sec. 4) conserve momentum and energy."""
    import numpy as np
    rng = np.random.default_rng(0)
    for _ in range(20):
        mi, mj = rng.uniform(0.5, 5.0, 2)
        a, b = P.pair_ab(mi, mj)
        v, vs = rng.normal(size=3), rng.normal(size=3)
        g = v - vs
        sig = rng.normal(size=3)
        sig /= np.linalg.norm(sig)
        vp = v - a * g + a * np.linalg.norm(g) * sig
        vsp = v - a * g - b * np.linalg.norm(g) * sig
        assert np.allclose(mi * v + mj * vs, mi * vp + mj * vsp, atol=1e-13)
        assert mi * v @ v + mj * vs @ vs == pytest.approx(mi * vp @ vp + mj * vsp @ vsp, rel=1e-13)


def test_krook_wu_constants():
    """Sec. 6.1 constants; at m1 = m2 they reduce to mu = 1, p = 1/2, A = B = 1/4,
    so Q(t) = 1/(e^{t/4} - 1) and the solvability condition holds."""
    k = bkw.KrookWu(1.0, 1.0)
    assert (k.mu, k.p1, k.p2) == pytest.approx((1.0, 0.5, 0.5))
    assert (k.A, k.B) == pytest.approx((0.25, 0.25))
    assert k.Q(4.0) == pytest.approx(1.0 / (math.e - 1.0), rel=1e-14)
    assert k.K(4.0) == pytest.approx(1.0 - math.exp(-1.0), rel=1e-14)
    for r in (2.0, 4.0, 8.0):
        assert bkw.KrookWu(r, 1.0).condition == pytest.approx(0.0, abs=1e-15)


def test_krook_wu_derivative_by_finite_difference():
    """The printed df/dt agrees with a centred difference of the printed f."""
    import numpy as np
    k = bkw.KrookWu(2.0, 1.0)
    v2 = np.linspace(0.0, 9.0, 50)
    for i in (1, 2):
        h = 1e-5
        fd = (k.f(i, 4.0 + h, v2) - k.f(i, 4.0 - h, v2)) / (2 * h)
        assert np.allclose(k.dfdt(i, 4.0, v2), fd, rtol=1e-7, atol=1e-12)
