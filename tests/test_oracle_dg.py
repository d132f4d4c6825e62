"""Pins of the nodal DG slab oracle (Sec. 5): the GLL rule (including the K = 3 weights
the paper prints), the Lagrange derivative, exactness of the transport operator on
polynomials of the element degree, the discrete mass balance, the zero net flux
through a diffuse wall, and SSP-RK2 around it; the Maxwellian that builds the inflow
and wall states carries the density, velocity and temperature it is given."""
import numpy as np
import pytest

from oracle import dg, moments as Mo, spectral as S, stepping as T


@pytest.mark.parametrize("m,n,u,T,N,L", [
    (1.0, 1.0, (0.0, 0.0, 0.0), 1.0, 32, 6.0),
    (2.0, 0.7, (0.3, -0.2, 0.1), 0.5, 48, 6.0),
    (1.0, 1.3, (0.0, -0.3, 0.0), 1.7, 48, 8.0),
    (32.75, 0.9, (0.0, 0.0, 0.05), 1.0, 48, 6.0 * np.sqrt(1.0 / 32.75)),
])
def test_maxwellian_moments_are_its_parameters(m, n, u, T, N, L):
    """The nondimensional moments of Sec. 3 (n = int f, u = int v f / n,
    T = 2m/(3n) int |v - u|^2 f), taken by the rectangle rule on a grid that resolves
    the Maxwellian (spacing and box chosen so that the rule's error and the tails are
    below 1e-14), return the parameters it was built with.  A wrong normalisation
    (e.g. (m/(2 pi T))^{3/2}) or temperature convention (exp(-m v^2/(2T))) fails."""
    f = dg.maxwellian(N, L, m, n, u, T)
    mo = Mo.moments(f, m, L)
    assert abs(mo["n"] - n) <= 1e-12 * n
    np.testing.assert_allclose(mo["u"], u, rtol=0, atol=1e-12)
    assert abs(mo["T"] - T) <= 1e-12 * T


def test_gll_k3_is_the_printed_example():
    """Sec. 5.1: with K = 3 GLL points the diagonal of H on the standard element is
    (1/3, 4/3, 1/3), i.e. the GLL weights, at the points (-1, 0, 1)."""
    x, w = dg.gll(3)
    np.testing.assert_allclose(x, [-1.0, 0.0, 1.0], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)


@pytest.mark.parametrize("K", [2, 3, 4, 5, 6])
def test_gll_rule(K):
    """Weights sum to 2, the rule is exact to degree 2K - 3, K = 4 has the points
    +-1, +-1/sqrt(5) with weights 1/6, 5/6."""
    x, w = dg.gll(K)
    assert abs(w.sum() - 2.0) < 1e-14
    for p in range(2 * K - 2):
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        assert abs(np.sum(w * x ** p) - exact) < 1e-13
    if K == 4:
        np.testing.assert_allclose(x, [-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1], atol=1e-15)
        np.testing.assert_allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)


@pytest.mark.parametrize("K", [2, 3, 4, 5])
def test_lagrange_derivative_is_exact_on_polynomials(K):
    x, _ = dg.gll(K)
    D = dg.lagrange_derivative(x)
    rng = np.random.default_rng(K)
    c = rng.normal(size=K)                 # degree K - 1
    p = np.polynomial.Polynomial(c)
    # interpolant values at the nodes, derivative at the nodes: sum_m p(x_m) phi_m'(x_q)
    np.testing.assert_allclose(D @ p(x), p.deriv()(x), atol=1e-12)


def _slab(K, Ne, left, right, N=8, Ls=(3.0, 2.5), masses=(1.0, 2.0)):
    return dg.Slab(x0=-0.5, x1=0.5, Ne=Ne, K=K, masses=masses, N=N, Ls=Ls, left=left, right=right)


@pytest.mark.parametrize("K,Ne", [(2, 3), (3, 4), (4, 5)])
def test_transport_exact_on_element_degree_polynomials(K, Ne):
    """f(x, v) = p(x) g_i(v) with p of degree K - 1 and inflow states p(x0) g_i, p(x1) g_i:
    the DG operator gives -v_x p'(x) g_i(v) at every node exactly (integration by parts
    is exact under the GLL rule, and the upwind flux of a continuous f is its value)."""
    rng = np.random.default_rng(10 + K)
    p = np.polynomial.Polynomial(rng.uniform(0.5, 1.0, size=K) / np.arange(1, K + 1))
    masses, Ls, N = (1.0, 2.0), (3.0, 2.5), 8
    u, Tt = (0.2, -0.1, 0.0), 0.9
    g = [dg.maxwellian(N, Ls[i], masses[i], 1.0, u, Tt) for i in range(2)]
    left = dg.Boundary("inflow", u=u, T=Tt, n=(p(-0.5),) * 2)
    right = dg.Boundary("inflow", u=u, T=Tt, n=(p(0.5),) * 2)
    slab = _slab(K, Ne, left, right, N, Ls, masses)
    X = slab.node_positions()
    F = np.stack([np.stack([np.stack([p(X[e, m]) * g[i] for i in range(2)]) for m in range(K)])
                  for e in range(Ne)])
    got = slab.transport(F)
    for i in range(2):
        ref = -slab.vx(i)[None, None] * p.deriv()(X)[:, :, None, None, None] * g[i][None, None]
        np.testing.assert_allclose(got[:, :, i], ref, rtol=0, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("kinds", [("inflow", "inflow"), ("wall", "inflow"), ("wall", "wall")])
def test_mass_balance(kinds):
    """For any F the GLL-weighted total of the transport term equals the net inflow
    through the two ends (the interior fluxes cancel, the volume terms sum to zero);
    through a diffuse wall that net flow is zero by eq. bc_nwall."""
    rng = np.random.default_rng(3)
    mk = {"inflow": dg.Boundary("inflow", u=(0.3, 0, 0), T=1.1, n=(0.8, 0.5)),
          "wall": dg.Boundary("wall", u=(0.0, 0.2, 0.0), T=0.9)}
    slab = _slab(3, 4, mk[kinds[0]], mk[kinds[1]])
    F = rng.random((4, 3, 2, 8, 8, 8))
    dm = np.array([sum(slab.h / 2 * slab.w[m] * slab.transport(F)[e, m, i].sum() * (2 * slab.Ls[i] / 8) ** 3
                       for e in range(4) for m in range(3)) for i in range(2)])
    flux = slab.boundary_mass_flux(F)
    np.testing.assert_allclose(dm, flux, rtol=1e-12, atol=1e-12)
    if kinds == ("wall", "wall"):
        np.testing.assert_allclose(flux, 0.0, atol=1e-12)


def test_wall_density_matches_outgoing_flux():
    """Diffuse wall: the outside state is n_w times the wall Maxwellian, and the mass it
    carries in equals the mass the inside trace carries out."""
    rng = np.random.default_rng(4)
    bc = dg.Boundary("wall", u=(0.0, 0.1, 0.0), T=1.2)
    slab = _slab(2, 2, bc, bc)
    trace = rng.random((2, 8, 8, 8))
    ext = slab.exterior(bc, trace, +1.0)
    for i in range(2):
        vx = np.broadcast_to(slab.vx(i), trace[i].shape)
        out = np.sum(np.where(vx >= 0, vx * trace[i], 0))
        inn = np.sum(np.where(vx < 0, vx * ext[i], 0))
        assert abs(out + inn) < 1e-12 * out
        Mw = dg.maxwellian(8, slab.Ls[i], slab.masses[i], 1.0, bc.u, bc.T)
        ratio = ext[i] / Mw
        assert np.ptp(ratio) < 1e-12 * ratio.max()


def test_ssprk2_slab_step_mass_budget():
    """One SSP-RK2 step of transport + projected collisions from the inflow Maxwellian:
    the projection conserves each species' mass at every node, so the total changes
    only through the ends, by dt/2 (flux(F) + flux(F1)), F1 = F + dt L(F)."""
    masses, Ls, N = (1.0, 2.0), (5.0, 5.0), 16
    u, Tt, n = (0.1, 0.0, 0.0), 1.0, (1.0, 0.6)
    bc = dg.Boundary("inflow", u=u, T=Tt, n=n)
    slab = dg.Slab(x0=0.0, x1=1.0, Ne=2, K=2, masses=masses, N=N, Ls=Ls, left=bc, right=bc)
    f0 = np.stack([dg.maxwellian(N, Ls[i], masses[i], n[i], u, Tt) for i in range(2)])
    F = np.broadcast_to(f0, (2, 2) + f0.shape).copy()
    prob = S.vhs_problem(masses, 0.74, 5.0, N, 6, 8)
    rhs = dg.slab_rhs(slab, prob)
    dt = 0.01
    assert np.abs(slab.transport(F)).max() == 0.0          # uniform inflow state: no transport
    F1 = F + dt * rhs(F)
    F2 = T.ssprk2(F, rhs, dt, 1)
    budget = 0.5 * dt * (slab.boundary_mass_flux(F) + slab.boundary_mass_flux(F1))
    np.testing.assert_allclose(slab.mass(F2) - slab.mass(F), budget, rtol=1e-10, atol=1e-15)
