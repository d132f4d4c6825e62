"""The shifted field as a product of per-axis operators (the form the matrix-core gain
evaluates), checked against the spectral form of Sec. 4 on the CPU.

A(v) = sum_k f_hat_k e^{i theta.k} e^{i pi k.v/L} over the literal mode set (the DFT
index N/2 read as the mode -N/2) equals (R_x (x) R_y (x) R_z) f with
R(n, m) = (1/N) sum_l e^{i l (2 pi (n - m)/N + theta)}; R = C + i s u u^T with C
circulant, s = -sin(N theta / 2) / N, u = (-1)^n; and on each x-plane every term of
Re A and Im A other than C_x C_y C_z f and s_x u_x C_y C_z a_x is u_y b(z) + a(y) u_z.
The spectral side is the oracle's Fourier pair; the operator side is written here from
the definitions above."""
import numpy as np
import pytest

from oracle import spectral as OS


def _shift_matrix(N, theta):
    n = np.arange(N)
    l = OS.signed_modes(N)
    d = 2.0 * np.pi * (n[:, None] - n[None, :]) / N
    return np.exp(1j * (d[:, :, None] + theta) * l[None, None, :]).sum(axis=2) / N


def _fields(N, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((N, N, N)) + 2.0
    theta = rng.uniform(-1.3, 1.3, 3)
    return f, theta


@pytest.mark.parametrize("N,seed", [(8, 1), (12, 2), (16, 3)])
def test_separable_operator_equals_spectral_shift(N, seed):
    f, theta = _fields(N, seed)
    L = 6.0
    KX, KY, KZ = OS.mode_grids(N)
    A_spec = OS.synthesize(np.exp(1j * (theta[0] * KX + theta[1] * KY + theta[2] * KZ))
                           * OS.fourier_coefficients(f, L), L)
    R = [_shift_matrix(N, t) for t in theta]
    A_sep = np.einsum("ai,bj,ck,ijk->abc", R[0], R[1], R[2], f, optimize=True)
    assert np.abs(A_sep - A_spec).max() <= 1e-12 * np.abs(A_spec).max()


@pytest.mark.parametrize("N", [8, 12, 32])
def test_shift_matrix_is_circulant_plus_rank_one(N):
    theta = 0.77
    R = _shift_matrix(N, theta)
    C = R.real
    n = np.arange(N)
    c = C[:, 0]
    assert np.allclose(C, c[(n[:, None] - n[None, :]) % N], atol=1e-14)   # C(n, m) = c(n - m)
    u = (-1.0) ** n
    s = -np.sin(N * theta / 2) / N
    assert np.allclose(R.imag, s * np.outer(u, u), atol=1e-14)


@pytest.mark.parametrize("N,seed", [(8, 4), (12, 5)])
def test_plane_corrections_are_rank_two(N, seed):
    """Re A and Im A on each x-plane from T, s_x u_x P_x and two rank-one terms each."""
    f, theta = _fields(N, seed)
    R = [_shift_matrix(N, t) for t in theta]
    C = [r.real for r in R]
    n = np.arange(N)
    u = (-1.0) ** n
    s = [-np.sin(N * t / 2) / N for t in theta]
    A = np.einsum("ai,bj,ck,ijk->abc", R[0], R[1], R[2], f, optimize=True)
    Cx, Cy, Cz = C
    sx, sy, sz = s
    T = np.einsum("ai,bj,ck,ijk->abc", Cx, Cy, Cz, f, optimize=True)
    a_x = np.einsum("i,ijk->jk", u, f)              # alternating sums over the axes named
    a_y = np.einsum("j,ijk->ik", u, f)
    a_z = np.einsum("k,ijk->ij", u, f)
    a_xy = np.einsum("i,j,ijk->k", u, u, f)
    a_xz = np.einsum("i,k,ijk->j", u, u, f)
    a_yz = np.einsum("j,k,ijk->i", u, u, f)
    a_xyz = np.einsum("i,j,k,ijk->", u, u, u, f)
    P_x = Cy @ a_x @ Cz.T                              # C_y C_z a_x, [y][z]
    P_y = Cx @ a_y @ Cz.T                              # C_x C_z a_y, [x][z]
    P_z = Cx @ a_z @ Cy.T                              # C_x C_y a_z, [x][y]
    L_xy, L_xz, L_yz = Cz @ a_xy, Cy @ a_xz, Cx @ a_yz
    for x in range(N):
        ux = u[x]
        b_re = -(sx * sy * ux * L_xy + sy * sz * u * L_yz[x])
        a_re = -sx * sz * ux * L_xz
        b_im = sy * P_y[x] - sx * sy * sz * ux * u * a_xyz
        a_im = sz * P_z[x]
        re = T[x] + np.outer(u, b_re) + np.outer(a_re, u)
        im = sx * ux * P_x + np.outer(u, b_im) + np.outer(a_im, u)
        scale = np.abs(A).max()
        assert np.abs(re - A[x].real).max() <= 1e-12 * scale
        assert np.abs(im - A[x].imag).max() <= 1e-12 * scale
