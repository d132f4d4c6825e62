"""The kernel mode of the variable-soft-sphere kernel, alpha in (1, 2] (oracle; test
infrastructure).

Sec. 2 (eq. VSS, and its dimensionless form NVSS) gives B_ij = C |g|^gamma (1 + cos chi)^{alpha-1}
with cos chi = sigma . g_hat and gamma = 2(1 - omega).  The fast method of Sec. 4 needs,
below eq. GG,

    F(k, rho, sigma) = rho^2 int_{S^2} B(rho, sigma . g_hat) e^{-i pi rho a k . g_hat / L} dg_hat,

which for alpha > 1 depends on sigma (through mu = sigma . k_hat) and is complex, so the
sum over sigma can no longer be taken before the transform.

Evaluation: put the pole of the g_hat sphere at sigma, g_hat = t sigma + sqrt(1 - t^2) e(phi)
with e(phi) a unit vector orthogonal to sigma.  Then k_hat . g_hat = t mu + sqrt(1 - t^2)
sqrt(1 - mu^2) cos(phi - phi0), and the azimuthal integral of the plane wave is
2 pi J0(z sqrt(1 - t^2) sqrt(1 - mu^2)), z = pi rho a |k| / L.  Hence

    F = 2 pi C rho^{gamma+2} int_{-1}^{1} (1 + t)^{alpha-1} e^{-i z mu t} J0(z sqrt((1-t^2)(1-mu^2))) dt.

The factor (1 + t)^{alpha-1} is the Gauss-Jacobi weight (beta = alpha - 1), so it is
integrated exactly; the rest is an entire function of t that oscillates at frequency z,
so the number of nodes grows with z.

The loss weight needs only int_{S^2} (1 + sigma . g_hat)^{alpha-1} dsigma = 2 pi 2^alpha / alpha,
so G-(m) for alpha > 1 is the alpha = 1 weight times 2^{alpha-1} / alpha.
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.special


def sphere_weight_integral(alpha: float) -> float:
    """int_{S^2} (1 + sigma . g_hat)^{alpha-1} dsigma = 2 pi int_{-1}^{1} (1+t)^{alpha-1} dt."""
    return 2.0 * np.pi * 2.0 ** alpha / alpha


def _nodes(n: int, alpha: float):
    return scipy.special.roots_jacobi(n, 0.0, alpha - 1.0)


def _integral(z: np.ndarray, mu: np.ndarray, alpha: float, n: int) -> np.ndarray:
    t, w = _nodes(n, alpha)
    zt = z[:, None]
    mt = mu[:, None]
    arg = zt * np.sqrt(np.clip((1.0 - t * t)[None, :] * (1.0 - mt * mt), 0.0, None))
    vals = np.exp(-1j * zt * mt * t[None, :]) * scipy.special.j0(arg)
    return vals @ w


def nodes_for(z: float) -> int:
    """Gauss-Jacobi nodes for an integrand that oscillates at frequency <= z: the rule
    with n nodes is exact to polynomial degree 2n - 1, and n = z + 32 leaves a wide margin
    (checked by doubling in the tests)."""
    return int(np.ceil(z)) + 32


def kernel_mode(kvec, rho: float, sigma, a: float, gamma: float, alpha: float, C: float, L: float,
                nodes=nodes_for) -> np.ndarray:
    """F(k, rho, sigma) for k given as signed mode vectors [..., 3] (complex, shape [...]).
    Modes are grouped by z in bins of width 8, each integrated with nodes(bin's largest z)."""
    kvec = np.asarray(kvec, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    shape = kvec.shape[:-1]
    kv = kvec.reshape(-1, 3)
    kabs = np.linalg.norm(kv, axis=1)
    mu = np.zeros_like(kabs)
    nz = kabs > 0
    mu[nz] = (kv[nz] @ sigma) / kabs[nz]
    z = np.pi * rho * a * kabs / L
    out = np.empty(z.shape, dtype=np.complex128)
    bins = np.floor(z / 8.0).astype(int)
    for bn in np.unique(bins):
        sel = bins == bn
        out[sel] = _integral(z[sel], mu[sel], alpha, nodes(8.0 * (bn + 1)))
    return (2.0 * np.pi * C * rho ** (gamma + 2.0) * out).reshape(shape)


@functools.lru_cache(maxsize=800)
def _grid_cached(N: int, rho: float, sigma: tuple, a: float, gamma: float, alpha: float, C: float,
                 L: float) -> np.ndarray:
    j = np.arange(N)
    m = np.where(j < N // 2, j, j - N).astype(np.float64)
    kvec = np.stack(np.meshgrid(m, m, m, indexing="ij"), axis=-1)
    F = kernel_mode(kvec, rho, np.array(sigma), a, gamma, alpha, C, L)
    F.flags.writeable = False
    return F


def kernel_mode_grid(N: int, rho: float, sigma, a: float, gamma: float, alpha: float, C: float,
                     L: float) -> np.ndarray:
    """F at every mode of the N^3 grid (DFT index order), remembered across calls: the
    same pair and quadrature point recur for every spatial point and time step."""
    return _grid_cached(int(N), float(rho), tuple(float(x) for x in sigma), float(a), float(gamma), float(alpha),
                        float(C), float(L))
