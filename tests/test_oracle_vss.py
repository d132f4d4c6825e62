"""Pins of the oracle's VSS kernel mode (alpha > 1) and of the operator built on it.

F(k, rho, sigma) is checked against closed forms at alpha = 1 and alpha = 2, against a
brute-force quadrature of its defining sphere integral, and for the symmetries it must
have; the operator against the O(N^6) direct sum and against two moment identities of
Maxwell molecules (gamma = 0) that hold for any distribution and fix the angular
structure of the kernel: the momentum exchanged between species and the relaxation of
the shear stress of one species."""
import numpy as np
import pytest
import scipy.special

from oracle import quadrature as Qd, spectral as S, vss as V
from synth import inputs as I


def _ref_F_alpha1(kvec, rho, a, gamma, C, L):
    z = np.pi * rho * a * np.linalg.norm(kvec, axis=-1) / L
    return 4 * np.pi * C * rho ** (gamma + 2) * np.sinc(z / np.pi)


def _rand_k(rng, n, kmax=16):
    return rng.integers(-kmax, kmax, size=(n, 3)).astype(float)


def _unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def test_alpha_one_is_the_vhs_mode():
    """alpha = 1: (1 + cos chi)^0 = 1 and F reduces to 4 pi C rho^{gamma+2} sinc(z)."""
    rng = np.random.default_rng(0)
    k = _rand_k(rng, 200)
    for rho, a in ((0.7, 0.5), (3.1, 2 / 3), (5.0, 0.97)):
        got = V.kernel_mode(k, rho, _unit(rng), a, 0.52, 1.0, 1.3, 6.0)
        ref = _ref_F_alpha1(k, rho, a, 0.52, 1.3, 6.0)
        np.testing.assert_allclose(got, ref, rtol=0, atol=3e-13 * np.abs(ref).max())


def test_alpha_two_closed_form():
    """alpha = 2: the kernel factor 1 + sigma.g_hat has Legendre components P0 + P1, so by
    the Funk-Hecke formula F = 4 pi C rho^{gamma+2} [j0(z) - i mu j1(z)], mu = sigma.k_hat."""
    rng = np.random.default_rng(1)
    k = _rand_k(rng, 300)
    k = k[np.linalg.norm(k, axis=1) > 0]
    for rho, a in ((0.9, 0.5), (4.2, 1 / 3)):
        sg = _unit(rng)
        got = V.kernel_mode(k, rho, sg, a, 0.4, 2.0, 0.8, 5.0)
        kab = np.linalg.norm(k, axis=1)
        z = np.pi * rho * a * kab / 5.0
        mu = (k @ sg) / kab
        ref = 4 * np.pi * 0.8 * rho ** 2.4 * (scipy.special.spherical_jn(0, z)
                                               - 1j * mu * scipy.special.spherical_jn(1, z))
        np.testing.assert_allclose(got, ref, rtol=0, atol=3e-13 * np.abs(ref).max())


def test_brute_force_sphere_quadrature():
    """alpha = 1.4: the defining integral over g_hat taken with a product rule about the
    z axis (not aligned with sigma), against the pole-at-sigma reduction."""
    rng = np.random.default_rng(2)
    G, W = Qd.product_sphere_rule(400)
    k = _rand_k(rng, 12, kmax=8)
    rho, a, gamma, C, L, alpha = 1.7, 0.6, 0.38, 1.1, 6.0, 1.4
    for _ in range(3):
        sg = _unit(rng)
        got = V.kernel_mode(k, rho, sg, a, gamma, alpha, C, L)
        h = (1.0 + G @ sg) ** (alpha - 1.0)
        ph = np.exp(-1j * np.pi * rho * a * (k @ G.T) / L)
        ref = C * rho ** (gamma + 2) * (ph * h[None, :]) @ W
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-7 * np.abs(ref).max())


def test_symmetries():
    """F(-k) = conj F(k), F(k, -sigma) = conj F(k, sigma) and F(R k, R sigma) = F(k, sigma)
    for a rotation R; F(0) = C rho^{gamma+2} 2 pi 2^alpha / alpha."""
    rng = np.random.default_rng(3)
    k = _rand_k(rng, 100)
    sg = _unit(rng)
    args = (2.3, 0.45, 0.3, 1.36, 0.9, 6.0)
    rho, a, gamma, alpha, C, L = args
    F = V.kernel_mode(k, rho, sg, a, gamma, alpha, C, L)
    np.testing.assert_allclose(V.kernel_mode(-k, rho, sg, a, gamma, alpha, C, L), F.conj(), atol=1e-14)
    np.testing.assert_allclose(V.kernel_mode(k, rho, -sg, a, gamma, alpha, C, L), F.conj(), atol=1e-14)
    Rm = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    Fr = V.kernel_mode(k @ Rm.T, rho, Rm @ sg, a, gamma, alpha, C, L)
    np.testing.assert_allclose(Fr, F, atol=1e-13)
    F0 = V.kernel_mode(np.zeros((1, 3)), rho, sg, a, gamma, alpha, C, L)[0]
    assert abs(F0 - C * rho ** (gamma + 2) * 2 * np.pi * 2 ** alpha / alpha) < 1e-13 * abs(F0)


def test_funk_hecke_series():
    """A second route: F = C rho^{gamma+2} sum_l (2l+1) (-i)^l lambda_l j_l(z) P_l(mu) with
    lambda_l = 2 pi int (1+t)^{alpha-1} P_l(t) dt taken by adaptive quadrature."""
    import scipy.integrate
    rng = np.random.default_rng(4)
    k = _rand_k(rng, 40, kmax=6)
    k = k[np.linalg.norm(k, axis=1) > 0]
    rho, a, gamma, alpha, C, L = 1.2, 0.5, 0.4, 1.32, 1.0, 6.0
    sg = _unit(rng)
    kab = np.linalg.norm(k, axis=1)
    z = np.pi * rho * a * kab / L
    mu = (k @ sg) / kab
    lmax = int(z.max()) + 40
    lam = [2 * np.pi * scipy.integrate.quad(lambda t, l=l: (1 + t) ** (alpha - 1) * scipy.special.eval_legendre(l, t),
                                            -1, 1, limit=400, epsabs=1e-15, epsrel=1e-13)[0]
           for l in range(lmax)]
    ser = sum((2 * l + 1) * (-1j) ** l * lam[l] * scipy.special.spherical_jn(l, z) * scipy.special.eval_legendre(l, mu)
              for l in range(lmax))
    ref = C * rho ** (gamma + 2) * ser
    got = V.kernel_mode(k, rho, sg, a, gamma, alpha, C, L)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_loss_weight_scale_at_zero():
    """G-(0) = C R^{gamma+3}/(gamma+3) x 4 pi x 2 pi 2^alpha / alpha."""
    R, gamma, C, L, alpha = 4.0, 0.4, 1.2, 6.0, 1.36
    got = S.loss_weight(np.array([0.0]), R, gamma, C, L, alpha=alpha)[0]
    ref = C * R ** (gamma + 3) / (gamma + 3) * 4 * np.pi * 2 * np.pi * 2 ** alpha / alpha
    assert abs(got - ref) < 1e-13 * ref


def test_fast_equals_direct_sum_vss():
    """N = 4, alpha = 1.36 and 2: the FFT evaluation of Sec. 4 equals the explicit double
    sum of eq. (sum) with the same sigma-dependent weights."""
    rng = np.random.default_rng(5)
    N, L = 4, 5.0
    sig, ws = Qd.design_quadrature(6)
    for alpha in (1.36, 2.0):
        pr = S.make_pair(1.0, 2.0, 0.8, 0.7, L, 3, sig, ws, alpha=alpha)
        fi = rng.random((N, N, N))
        fj = rng.random((N, N, N))
        fast = S.collide_pair_fast(fi, fj, pr)
        direct = S.collide_pair_direct(fi, fj, pr)
        np.testing.assert_allclose(fast, direct, rtol=0, atol=1e-12 * np.abs(direct).max())


def _gaussian(N, L, n, u, cov):
    v = I.velocity_grid(N, L)
    X = np.stack(np.meshgrid(v, v, v, indexing="ij"), -1) - np.asarray(u)
    ic = np.linalg.inv(cov)
    e = np.einsum("...i,ij,...j->...", X, ic, X)
    return n * np.exp(-0.5 * e) / np.sqrt((2 * np.pi) ** 3 * np.linalg.det(cov))


# N = 24 on L = 6 with the 24-point design and 12 radial points resolves these inputs:
# the identities then hold to about 1e-3 (the truncation of g at R and the sphere rule).
N_M, L_M, M_M, NRHO_M = 24, 6.0, 24, 12


def _maxwell_pair(mi, mj, alpha, C=1.0):
    sig, ws = Qd.design_quadrature(M_M)
    return S.make_pair(mi, mj, 1.0, C, L_M, NRHO_M, sig, ws, alpha=alpha)


def _velocity_moment(Q, powers):
    v = I.velocity_grid(N_M, L_M)
    w = [v ** p for p in powers]
    return np.einsum("ijk,i,j,k->", Q, *w) * (2 * L_M / N_M) ** 3


@pytest.mark.parametrize("alpha", [1.0, 1.36])
def test_maxwell_momentum_exchange(alpha):
    """Maxwell molecules (omega = 1): int v Q^{ij} dv = -a C kappa1 n_i n_j (u_i - u_j) with
    kappa1 = int (1 + cos chi)^{alpha-1} (1 - cos chi) dsigma = 2 pi 2^{alpha+1}/(alpha(alpha+1)),
    for any f^i, f^j (here two drifting Gaussians of different temperatures, m = (1, 2))."""
    pr = _maxwell_pair(1.0, 2.0, alpha)
    ui, uj = np.array([0.3, -0.2, 0.1]), np.array([-0.2, 0.25, 0.0])
    fi = _gaussian(N_M, L_M, 1.0, ui, np.eye(3) * 0.4)
    fj = _gaussian(N_M, L_M, 0.7, uj, np.eye(3) * 0.25)
    Q = S.collide_pair_fast(fi, fj, pr)
    mom = np.array([_velocity_moment(Q, p) for p in ((1, 0, 0), (0, 1, 0), (0, 0, 1))])
    kappa1 = 2 * np.pi * 2 ** (alpha + 1) / (alpha * (alpha + 1))
    ref = -pr.a * kappa1 * 1.0 * 0.7 * (ui - uj)
    print(f"alpha={alpha}: relative error {np.abs(mom - ref).max() / np.abs(ref).max():.2e}")
    np.testing.assert_allclose(mom, ref, rtol=0, atol=1e-3 * np.abs(ref).max())


@pytest.mark.parametrize("alpha", [1.0, 1.4])
def test_maxwell_shear_relaxation(alpha):
    """Maxwell molecules, one species: int v_x v_y Q(f, f) dv = -(3/4) C kappa2 n P_xy with
    kappa2 = int (1 + cos chi)^{alpha-1} sin^2 chi dsigma = 2 pi 2^{alpha+2}/((alpha+1)(alpha+2))
    and P_xy = n cov_xy for a sheared Gaussian."""
    pr = _maxwell_pair(1.0, 1.0, alpha)
    cov = 0.5 * np.array([[0.9, 0.3, 0.0], [0.3, 0.7, 0.1], [0.0, 0.1, 0.8]])
    f = _gaussian(N_M, L_M, 1.0, (0.0, 0.0, 0.0), cov)
    Q = S.collide_pair_fast(f, f, pr)
    got = _velocity_moment(Q, (1, 1, 0))
    kappa2 = 2 * np.pi * 2 ** (alpha + 2) / ((alpha + 1) * (alpha + 2))
    ref = -0.75 * kappa2 * 1.0 * cov[0, 1]
    print(f"alpha={alpha}: relative error {abs(got / ref - 1):.2e}")
    assert abs(got - ref) < 3e-3 * abs(ref)


def test_node_rule_is_converged():
    """At the largest z of an N = 48 grid (a = 0.97, rho = R of L = 6) doubling the
    Gauss-Jacobi nodes changes F by less than 1e-13 of F(0)."""
    rng = np.random.default_rng(6)
    k = _rand_k(rng, 400, kmax=24)
    sg = _unit(rng)
    args = (5.5, 0.97, 0.38, 1.36, 1.0, 6.0)
    rho, a, gamma, alpha, C, L = args
    F1 = V.kernel_mode(k, rho, sg, a, gamma, alpha, C, L)
    F2 = V.kernel_mode(k, rho, sg, a, gamma, alpha, C, L, nodes=lambda z: 2 * V.nodes_for(z))
    F0 = abs(V.kernel_mode(np.zeros((1, 3)), rho, sg, a, gamma, alpha, C, L)[0])
    assert np.abs(F1 - F2).max() < 1e-13 * F0
