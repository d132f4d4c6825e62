"""Pins of the species-specific grid reading (oracle): the interpolant passes through
the samples where two grids coincide, reproduces trigonometric polynomials exactly,
vanishes outside the source box, reduces to the single-grid operator when all boxes
agree, and carries a resolved heavy species onto the wide grid as if sampled there."""
import numpy as np
import pytest

from oracle import grids as G, moments as OM, spectral as S
from synth import inputs as I


@pytest.mark.parametrize("N", [8, 12])
def test_equal_boxes_give_the_samples(N):
    rng = np.random.default_rng(0)
    f = rng.random((N, N, N))
    assert np.abs(G.interpolate(f, 1.7, 1.7) - f).max() <= 1e-13


@pytest.mark.parametrize("N", [8, 16])
def test_coincident_points_and_zero_outside(N):
    """Grid L and grid 2L share every other point of the narrow grid: narrow -> wide
    returns those samples and zero outside [-L, L); wide -> narrow returns the wide
    samples at the shared points."""
    rng = np.random.default_rng(1)
    L = 1.5
    f = rng.random((N, N, N))
    g = G.interpolate(f, L, 2 * L)
    q = N // 4                                   # wide index of -L
    inner = slice(q, q + N // 2)
    np.testing.assert_allclose(g[inner, inner, inner], f[0::2, 0::2, 0::2], rtol=0, atol=1e-13)
    mask = np.zeros(N, bool)
    mask[inner] = True
    outside = ~(mask[:, None, None] & mask[None, :, None] & mask[None, None, :])
    assert np.all(g[outside] == 0.0)
    w = rng.random((N, N, N))
    h = G.interpolate(w, 2 * L, L)
    np.testing.assert_allclose(h[0::2, 0::2, 0::2], w[inner, inner, inner], rtol=0, atol=1e-13)


def _trig_poly(N, L, rng):
    """A real trigonometric polynomial on [-L, L)^3 with modes |k_d| < N/2 plus the
    Nyquist cosine along x; returns a callable of the three coordinate arrays."""
    modes = [tuple(rng.integers(-N // 2 + 1, N // 2, size=3)) for _ in range(6)]
    amps = rng.normal(size=6) + 1j * rng.normal(size=6)
    cn = rng.normal()

    def p(x, y, z):
        out = np.zeros(np.broadcast(x, y, z).shape)
        for (a, b, c), A in zip(modes, amps):
            out += 2 * (A * np.exp(1j * np.pi * (a * x + b * y + c * z) / L)).real
        out += cn * np.cos(np.pi * (N // 2) * x / L)
        return out
    return p


@pytest.mark.parametrize("N,L_from,L_to", [(8, 1.0, 2.3), (12, 2.0, 0.7), (16, 1.0484, 6.0)])
def test_trigonometric_polynomials_are_reproduced(N, L_from, L_to):
    rng = np.random.default_rng(N)
    p = _trig_poly(N, L_from, rng)
    vs = G.grid_points(N, L_from)
    X, Y, Z = np.meshgrid(vs, vs, vs, indexing="ij")
    f = p(X, Y, Z)
    got = G.interpolate(f, L_from, L_to)
    vt = G.grid_points(N, L_to)
    X, Y, Z = np.meshgrid(vt, vt, vt, indexing="ij")
    inside = ((X >= -L_from) & (X < L_from) & (Y >= -L_from) & (Y < L_from) & (Z >= -L_from) & (Z < L_from))
    ref = np.where(inside, p(X, Y, Z), 0.0)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(f).max()


def test_nyquist_in_two_dimensions_stays_a_product_of_cosines():
    """cos(pi N x / 2L) cos(pi N y / 2L) is reproduced exactly: the Nyquist mode is split
    evenly in each dimension (the literal -N/2 series would give cos(a + b) instead)."""
    N, L_from, L_to = 8, 1.0, 1.37
    vs = G.grid_points(N, L_from)
    c = np.cos(np.pi * (N // 2) * vs / L_from)
    f = c[:, None, None] * c[None, :, None] * np.ones(N)[None, None, :]
    vt = G.grid_points(N, L_to)
    inside = (vt >= -L_from) & (vt < L_from)
    ct = np.where(inside, np.cos(np.pi * (N // 2) * vt / L_from), 0.0)
    ref = ct[:, None, None] * ct[None, :, None] * inside[None, None, :]
    assert np.abs(G.interpolate(f, L_from, L_to) - ref).max() <= 1e-13


def test_equal_boxes_reduce_to_the_single_grid_operator():
    masses = (1.0, 2.0)
    prob = S.vhs_problem(masses, 0.74, 5.0, 8, 6, 4)
    f = I.draw_bimaxwellian_batch(np.random.default_rng(2), 1, 2, 8, 5.0, masses)[0]
    a = G.collide(f, prob, (5.0, 5.0))
    b = S.collide(f, prob)
    assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max()


def test_resolved_heavy_species_matches_direct_sampling_on_the_wide_grid():
    """m = (1, 32.75), L = (6, 6 sqrt(1/32.75)), N = 32: the heavy Maxwellian is resolved on
    its own grid, so its interpolant at the wide points equals the Maxwellian sampled there
    (to the spectral error), and the light species' collision term equals the single-grid
    one computed from that direct sampling."""
    N, M, nrho = 32, 6, 6
    masses = (1.0, 32.75)
    Ls = (6.0, 6.0 * np.sqrt(1.0 / 32.75))
    m1 = I.maxwellian(N, Ls[0], masses[0], 1.0, (0.0, 0.0, 0.0), 1.0)
    m2_narrow = I.maxwellian(N, Ls[1], masses[1], 0.8, (0.0, 0.0, 0.0), 1.1)
    m2_wide = I.maxwellian(N, Ls[0], masses[1], 0.8, (0.0, 0.0, 0.0), 1.1)
    g = G.interpolate(m2_narrow, Ls[1], Ls[0])
    assert np.abs(g - m2_wide).max() <= 1e-7 * m2_wide.max()
    prob = S.vhs_problem(masses, 0.5, Ls[0], N, M, nrho)
    f = np.stack([m1, m2_narrow])
    Q = G.collide_pairs(f, prob, Ls)
    ref = S.collide_pair_fast(m1, m2_wide, prob.pair(0, 1))
    assert np.abs(Q[0, 1] - ref).max() <= 1e-6 * np.abs(ref).max()
    # the pair (2, 2) runs on the narrow grid with R and the tables of that box
    prob2 = S.vhs_problem(masses, 0.5, Ls[1], N, M, nrho)
    ref22 = S.collide_pair_fast(m2_narrow, m2_narrow, prob2.pair(1, 1))
    assert np.abs(Q[1, 1] - ref22).max() <= 1e-14 * np.abs(ref22).max()


def test_projection_on_species_grids_conserves():
    masses = (1.0, 32.75)
    Ls = (6.0, 6.0 * np.sqrt(1.0 / 32.75))
    rng = np.random.default_rng(3)
    f = np.stack([I.maxwellian(16, Ls[0], masses[0], 1.0, (0.1, 0.0, 0.0), 1.0),
                  I.maxwellian(16, Ls[1], masses[1], 0.7, (0.0, 0.0, 0.0), 1.2)])
    prob = S.vhs_problem(masses, 0.5, Ls[0], 16, 6, 4)
    Q = G.collide(f, prob, Ls) + 1e-3 * rng.normal(size=f.shape)
    Qc = OM.conserve(Q, masses, Ls)
    assert np.all(OM.conservation_residual(Qc, masses, Ls) <= 1e-12)
