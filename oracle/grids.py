"""Species-specific velocity grids (oracle; test infrastructure).

Sec. 4, in the remark after eq. (domain), observes that one common domain becomes very
large for large mass ratios and names an independent velocity grid per species as a
remedy, which the paper leaves for later.  The reading implemented here:

* species i lives on its own grid v_n = -L_i + n 2L_i/N (same N for every species);
* the ordered pair (i, j) is evaluated by the single-grid method of Sec. 4 on the grid of
  half-width L_ij = max(L_i, L_j), with R_ij and every table taken for that L_ij;
* a species whose own box is narrower than L_ij is carried onto that grid by its own
  trigonometric interpolant (the truncated Fourier series of Sec. 4 on its box), taken
  as zero at points outside its box [-L_i, L_i) in any coordinate;
* Q^{ij}, computed on the L_ij grid, is carried back onto grid i by the interpolant of
  that grid (all points of the narrower grid i lie inside the wider box);
* Q^i = sum_j Q^{ij}; the conservation projection then runs on the species' own grids.

The interpolant of f on grid L is the real trigonometric interpolant
p(v) = sum_k f_hat_k c_{k_x}(v_x) c_{k_y}(v_y) c_{k_z}(v_z), with f_hat the coefficients of
Sec. 4 (modes k in [-N/2, N/2-1]), c_k(x) = e^{i pi k x / L} for |k| < N/2 and
c_{-N/2}(x) = cos(pi N x / (2L)): the Nyquist mode split evenly between +N/2 and -N/2 in
each dimension.  It agrees with the series at the grid points, is real for real data and
is a product of one-dimensional maps.
"""
from __future__ import annotations

import numpy as np

from . import spectral as S


def grid_points(N: int, L: float) -> np.ndarray:
    return -L + np.arange(N) * (2.0 * L / N)


def _evaluation_matrix(N: int, L_from: float, L_to: float) -> np.ndarray:
    """E[n, j] = c_{k_j}(v_n) at the target points v_n of the grid L_to, with k_j the signed
    mode of DFT index j (the Nyquist column a cosine); rows of points outside the source
    box are zero."""
    v = grid_points(N, L_to)
    k = S.signed_modes(N)
    E = np.exp(1j * np.pi * np.outer(v, k) / L_from)
    E[:, N // 2] = np.cos(np.pi * (N // 2) * v / L_from)
    inside = (v >= -L_from) & (v < L_from)
    return E * inside[:, None]


def interpolate(f: np.ndarray, L_from: float, L_to: float) -> np.ndarray:
    """Values on grid L_to of the trigonometric interpolant of f given on grid L_from."""
    N = f.shape[0]
    fhat = S.fourier_coefficients(f, L_from)       # explicit DFT matrices, DFT index order
    E = _evaluation_matrix(N, L_from, L_to)
    return np.einsum("ai,bj,ck,ijk->abc", E, E, E, fhat, optimize=True).real


def pair_grid(Ls, i: int, j: int) -> float:
    return max(Ls[i], Ls[j])


def collide_pairs(f: np.ndarray, prob, Ls, method: str = "fast") -> np.ndarray:
    """Q^{ij} for every ordered pair with species-specific grids: f [s][N][N][N] with
    species i on grid Ls[i]; result [s][s][N][N][N] with row i on grid Ls[i]."""
    fn = {"fast": S.collide_pair_fast, "direct": S.collide_pair_direct}[method]
    s = prob.s
    out = np.zeros((s, s) + f.shape[1:])
    for i in range(s):
        for j in range(s):
            Lij = pair_grid(Ls, i, j)
            fi = f[i] if Ls[i] == Lij else interpolate(f[i], Ls[i], Lij)
            fj = f[j] if Ls[j] == Lij else interpolate(f[j], Ls[j], Lij)
            omega, alpha, C = prob.kernel[i][j]
            pr = S.make_pair(prob.masses[i], prob.masses[j], omega, C, Lij, prob.nrho, prob.sigma,
                             prob.wsigma, alpha=alpha)
            q = fn(fi, fj, pr)
            out[i, j] = q if Ls[i] == Lij else interpolate(q, Lij, Ls[i])
    return out


def collide(f: np.ndarray, prob, Ls, method: str = "fast") -> np.ndarray:
    """Q^i = sum_j Q^{ij} with species-specific grids."""
    return collide_pairs(f, prob, Ls, method).sum(axis=1)
