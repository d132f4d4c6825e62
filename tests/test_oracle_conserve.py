"""Pins of the FP64 conservation projection and the moment formulas."""
import numpy as np
import pytest

from oracle import moments as Mo
from synth import inputs as I


def test_moments_of_maxwellian():
    """Sec. 3 moments of a well-resolved Maxwellian return its parameters."""
    N, L, m = 48, 6.0, 2.0
    f = I.maxwellian(N, L, m, 0.8, (0.3, -0.2, 0.1), 1.2)
    mo = Mo.moments(f, m, L)
    assert mo["n"] == pytest.approx(0.8, rel=1e-12)
    assert np.allclose(mo["u"], (0.3, -0.2, 0.1), atol=1e-12)
    assert mo["T"] == pytest.approx(1.2, rel=1e-12)


def _raw_q(seed, s=2, N=12):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(s, N, N, N))


@pytest.mark.parametrize("Ls", [(6.0, 6.0), (6.0, 1.0484)])
def test_projection_conserves(Ls):
    masses = (1.0, 32.75) if Ls[1] != Ls[0] else (1.0, 2.0)
    Q = _raw_q(1)
    Qc = Mo.conserve(Q, masses, Ls)
    r = Mo.conservation_residual(Qc, masses, Ls)
    assert np.all(r < 1e-14), r
    assert np.all(Mo.conservation_residual(Q, masses, Ls) > 1e-6)


def test_projection_is_orthogonal_and_idempotent():
    """Q~ = Q - A^T lam is the closest conserving field: the change lies in the row
    space of A and applying the projection twice changes nothing."""
    masses, Ls = (1.0, 2.0, 4.0), (6.0, 6.0, 6.0)
    Q = _raw_q(2, s=3)
    Qc = Mo.conserve(Q, masses, Ls)
    A = Mo.constraint_matrix(masses, Ls, Q.shape[1])
    d = (Q - Qc).reshape(-1)
    lam, *_ = np.linalg.lstsq(A.T, d, rcond=None)
    assert np.allclose(A.T @ lam, d, atol=1e-12 * np.abs(d).max())
    assert np.allclose(Mo.conserve(Qc, masses, Ls), Qc, atol=1e-14 * np.abs(Qc).max())


def test_projection_leaves_conserving_field_alone():
    """A field that already conserves (zero number, momentum and energy) is a fixed point:
    the difference of two same-grid Maxwellians with equal n, u and T moments projected
    onto the invariants is built here from an orthogonal complement."""
    masses, Ls, N = (1.0, 2.0), (6.0, 6.0), 10
    A = Mo.constraint_matrix(masses, Ls, N)
    rng = np.random.default_rng(3)
    x = rng.normal(size=A.shape[1])
    x -= A.T @ np.linalg.solve(A @ A.T, A @ x)         # any vector in the null space
    Q = x.reshape(2, N, N, N)
    assert np.allclose(Mo.conserve(Q, masses, Ls), Q, atol=1e-13 * np.abs(Q).max())


def test_invariant_rows_match_definitions():
    """Rows of A integrate number, m v and m |v|^2 with weight h^3 (rectangle rule)."""
    N, L = 8, 3.0
    A = Mo.constraint_matrix((1.0, 3.0), (L, L), N)
    one = np.ones((2, N, N, N))
    h3 = (2 * L / N) ** 3
    r = A @ one.ravel()
    assert r[0] == pytest.approx(N ** 3 * h3) and r[1] == pytest.approx(N ** 3 * h3)
    v = I.velocity_grid(N, L)
    assert r[2] == pytest.approx((1.0 + 3.0) * h3 * N * N * v.sum())
    assert r[5] == pytest.approx((1.0 + 3.0) * h3 * 3 * N * N * (v ** 2).sum())
