"""The Fourier spectral collision operator, written out plainly in FP64
(oracle; test infrastructure).

Everything follows Sec. 4 of the paper:

* truncated Fourier series on D_L = [-L, L]^3 with modes k in [-N/2, N/2-1]^3,
  f_hat_k = (2L)^{-3} int f e^{-i pi k.v/L} dv, evaluated by the rectangle rule on
  the grid v_n = -L + n 2L/N (which is exact for the trigonometric polynomial);
* the Galerkin-projected operator, eq. (sum): Q_hat_k = sum_{l+m=k} G(l,m) f_hat^i_l f_hat^j_m;
* the gain weight in quadrature form (below eq. GG),
  G+(l,m) = sum_{rho,sigma} w_rho w_sigma F(l+m, rho, sigma) e^{i pi rho (a l - b m).sigma / L};
* the kernel mode F (eq. below GG) and the loss weight G- (Sec. 4).

Readings where the paper leaves a choice (each one is listed with its reason in the
design notes of the repository):
* the sum over l + m = k is circular, l + m = k (mod N), which is what the FFT
  evaluation of the paper computes on the N^3 grid; F is evaluated at the wrapped
  output mode k;
* a DFT index j >= N/2 stands for the mode j - N, so index N/2 is the mode -N/2;
* the operator value at a grid point is the real part of the synthesised series.

For the VHS family (alpha = 1) the kernel is B = C |g|^gamma, gamma = 2(1 - omega);
then, with int_{S^2} e^{-i z k.g_hat} dg_hat = 4 pi sin(z|k|)/(z|k|),
    F(k, rho)  = 4 pi C rho^{gamma+2} sinc(pi a rho |k| / L)       (independent of sigma),
    G-(m)      = 16 pi^2 C int_0^R rho^{gamma+2} sinc(pi rho |m| / L) d rho,
where sinc(x) = sin(x)/x.  C is the pair prefactor, so Q^{ij} here already carries it.
For the VSS kernels (1 < alpha <= 2) F depends on sigma and is complex; it comes from
``vss.kernel_mode`` and G- carries the factor 2^{alpha-1}/alpha (see that module).

Three evaluations of the same discretised operator are provided:
* ``collide_pair_direct``: eq. (sum) as an explicit O(N^6) double loop with explicit
  Fourier matrices (no FFT anywhere), for tiny N;
* ``collide_pair_fast``: the fast algorithm of Sec. 4, the inner sum over l+m=k done
  as a convolution by FFT for every (rho, sigma);
* ``collide_pair_exact_sphere``: eq. (sum) with the sigma-integral done exactly,
  4 pi sinc(pi rho |a l - b m| / L), the M -> infinity limit of the sphere rule.
* ``collide_pair_dealiased``: eq. (sum) with l + m = k taken literally (no wrap-around,
  the Galerkin projection onto the kept modes), each sum a zero-padded convolution.
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np
import scipy.fft
import scipy.special

from . import params as P
from . import quadrature as Qd
from . import vss as V

# FFT worker threads: the host's CPU share (OMP_NUM_THREADS when set).
WORKERS = max(1, min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS") or (os.cpu_count() or 1))))


# --------------------------------------------------------------------------- modes
def signed_modes(N: int) -> np.ndarray:
    """Mode number of each DFT index: j for j < N/2, j - N otherwise."""
    j = np.arange(N)
    return np.where(j < N // 2, j, j - N)


def mode_grids(N: int):
    k = signed_modes(N)
    return np.meshgrid(k, k, k, indexing="ij")


def sinc(x):
    """sin(x)/x with sinc(0) = 1."""
    return np.sinc(np.asarray(x) / np.pi)


# ----------------------------------------------------- Fourier series (explicit)
def _fourier_matrix(N: int, L: float, sign: float) -> np.ndarray:
    v = -L + np.arange(N) * (2.0 * L / N)
    k = signed_modes(N)
    return np.exp(sign * 1j * np.pi * np.outer(k, v) / L)


def fourier_coefficients(f: np.ndarray, L: float) -> np.ndarray:
    """f_hat_k = N^{-3} sum_n f(v_n) e^{-i pi k.v_n/L}, indexed by DFT index."""
    N = f.shape[0]
    E = _fourier_matrix(N, L, -1.0) / N
    return np.einsum("ai,bj,ck,ijk->abc", E, E, E, f, optimize=True)


def synthesize(fhat: np.ndarray, L: float) -> np.ndarray:
    """sum_k f_hat_k e^{i pi k.v_n/L} at the grid points (complex)."""
    N = fhat.shape[0]
    E = _fourier_matrix(N, L, +1.0)  # [k, n]
    return np.einsum("ia,jb,kc,ijk->abc", E, E, E, fhat, optimize=True)


# ---------------------------------------------------------- kernel mode and loss
def kernel_mode_F(kabs, rho: float, a: float, gamma: float, C: float, L: float):
    """F(k, rho) = 4 pi C rho^{gamma+2} sinc(pi a rho |k| / L) for alpha = 1."""
    return 4.0 * np.pi * C * rho ** (gamma + 2.0) * sinc(np.pi * a * rho * np.asarray(kabs) / L)


def loss_weight(kabs, R: float, gamma: float, C: float, L: float, tol: float = 1e-14,
                alpha: float = 1.0) -> np.ndarray:
    """G-(m) = 16 pi^2 C int_0^R rho^{gamma+2} sinc(pi rho |m| / L) d rho, times
    2^{alpha-1}/alpha for a VSS kernel (the sigma integral of (1 + cos chi)^{alpha-1}
    over 4 pi).

    The radial integral uses Gauss-Jacobi quadrature for the weight rho^{gamma+2}
    (so the non-smooth factor rho^{gamma+2} is integrated exactly), doubling the
    number of points until two successive values agree to ``tol`` relative to
    int_0^R rho^{gamma+2} d rho (the size of the integrand)."""
    kabs = np.asarray(kabs, dtype=np.float64)
    flat = kabs.ravel()
    uniq, inv = np.unique(flat, return_inverse=True)

    def integral(n):
        x, w = scipy.special.roots_jacobi(n, 0.0, gamma + 2.0)
        rho = 0.5 * R * (1.0 + x)
        vals = sinc(np.pi * np.outer(uniq, rho) / L)
        return (0.5 * R) ** (gamma + 3.0) * (vals @ w)

    scale = R ** (gamma + 3.0) / (gamma + 3.0)
    n = 32
    prev = integral(n)
    while True:
        n *= 2
        cur = integral(n)
        if np.max(np.abs(cur - prev)) <= tol * scale:
            break
        if n >= 1024:
            raise RuntimeError("loss-weight quadrature did not converge")
        prev = cur
    sigma_factor = V.sphere_weight_integral(alpha) / (4.0 * np.pi)
    return (16.0 * np.pi ** 2 * C * sigma_factor * cur)[inv].reshape(kabs.shape)


# ------------------------------------------------------------------ pair set-up
@dataclass
class Pair:
    """Everything the operator needs for one ordered species pair (i, j)."""
    a: float
    b: float
    gamma: float
    C: float
    R: float
    L: float
    rho: np.ndarray      # radial Gauss-Legendre nodes on [0, R]
    wrho: np.ndarray
    sigma: np.ndarray    # (M, 3) sphere points
    wsigma: np.ndarray   # (M,)
    alpha: float = 1.0   # scattering parameter; > 1 for VSS

    def kernel_mode(self, kvec, q: int, p: int):
        """F(k, rho_q, sigma_p) at signed mode vectors kvec [..., 3]."""
        if self.alpha == 1.0:
            return kernel_mode_F(np.linalg.norm(kvec, axis=-1), self.rho[q], self.a, self.gamma, self.C, self.L)
        return V.kernel_mode(kvec, self.rho[q], self.sigma[p], self.a, self.gamma, self.alpha, self.C, self.L)

    def loss(self, kabs):
        return loss_weight(kabs, self.R, self.gamma, self.C, self.L, alpha=self.alpha)


def make_pair(mi: float, mj: float, omega: float, C: float, L: float, nrho: int,
              sigma: np.ndarray, wsigma: np.ndarray, R: float | None = None,
              alpha: float = 1.0) -> Pair:
    if not 1.0 <= alpha <= 2.0:
        raise ValueError("alpha must be in [1, 2]")
    a, b = P.pair_ab(mi, mj)
    if R is None:
        R = P.truncation_radius(L, mi, mj)
    rho, wrho = Qd.gauss_legendre(R, nrho)
    return Pair(a=a, b=b, gamma=P.gamma_exponent(omega), C=C, R=R, L=L, rho=rho, wrho=wrho,
                sigma=np.asarray(sigma, dtype=np.float64), wsigma=np.asarray(wsigma, dtype=np.float64),
                alpha=float(alpha))


# ------------------------------------------------------------------ direct sum
def _wrapped_output_modes(N, l_idx, m_idx):
    """DFT index of l + m (mod N) per dimension, and its signed mode."""
    kidx = (l_idx + m_idx) % N
    return kidx, signed_modes(N)[kidx]


def collide_pair_direct(fi: np.ndarray, fj: np.ndarray, pr: Pair, exact_sphere: bool = False,
                        linear: bool = False) -> np.ndarray:
    """Eq. (sum) evaluated as an explicit double sum over (l, m), O(N^6).

    G(l, m) = G+(l, m) - G-(m) with G+ in the (rho, sigma) quadrature form, or, when
    ``exact_sphere`` is set, with the sigma integral done in closed form.  With
    ``linear`` only pairs whose l + m lies in [-N/2, N/2-1]^3 contribute (no wrap)."""
    N = fi.shape[0]
    L = pr.L
    fhi = fourier_coefficients(fi, L).ravel()
    fhj = fourier_coefficients(fj, L).ravel()
    ks = signed_modes(N)
    idx = np.stack(np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij"), -1).reshape(-1, 3)
    modes = ks[idx]                                         # (N^3, 3) signed modes
    mabs = np.linalg.norm(modes, axis=1)
    Gminus = pr.loss(mabs)                                  # G-(m) for every m
    Qhat = np.zeros(N ** 3, dtype=np.complex128)
    rho, wrho = pr.rho, pr.wrho
    for li in range(N ** 3):
        kidx, kmode = _wrapped_output_modes(N, idx[li][None, :], idx)   # over all m
        kflat = (kidx[:, 0] * N + kidx[:, 1]) * N + kidx[:, 2]
        kabs = np.linalg.norm(kmode, axis=1)
        d = pr.a * modes[li][None, :] - pr.b * modes                      # a l - b m, (N^3, 3)
        Gplus = np.zeros(N ** 3, dtype=np.complex128)
        for q in range(len(rho)):
            if exact_sphere:
                if pr.alpha != 1.0:
                    raise ValueError("the closed-form sigma integral holds for alpha = 1 only")
                Fq = kernel_mode_F(kabs, rho[q], pr.a, pr.gamma, pr.C, L)
                ang = 4.0 * np.pi * sinc(np.pi * rho[q] * np.linalg.norm(d, axis=1) / L)
                Gplus += wrho[q] * Fq * ang
                continue
            for p in range(len(pr.wsigma)):
                Fqp = pr.kernel_mode(kmode, q, p)
                Gplus += wrho[q] * pr.wsigma[p] * Fqp * np.exp(1j * np.pi * rho[q] * (d @ pr.sigma[p]) / L)
        contrib = (Gplus - Gminus) * fhi[li] * fhj
        if linear:
            ksum = modes[li][None, :] + modes
            keep = np.all((ksum >= -(N // 2)) & (ksum <= N // 2 - 1), axis=1)
            contrib = np.where(keep, contrib, 0.0)
        np.add.at(Qhat, kflat, contrib)
    return synthesize(Qhat.reshape(N, N, N), L).real


def collide_pair_exact_sphere(fi, fj, pr: Pair) -> np.ndarray:
    """Eq. (sum) with the exact sigma integral (the M -> infinity limit)."""
    return collide_pair_direct(fi, fj, pr, exact_sphere=True)


# ------------------------------------------------------------------- fast sum
def _coefficients_fft(f: np.ndarray) -> np.ndarray:
    """f_hat_k via the FFT: the grid starts at -L, which contributes (-1)^{k1+k2+k3}."""
    N = f.shape[0]
    s = (-1.0) ** np.add.outer(np.add.outer(np.arange(N), np.arange(N)), np.arange(N))
    return s * scipy.fft.fftn(f, workers=WORKERS) / N ** 3


def _synthesize_fft(Qhat: np.ndarray) -> np.ndarray:
    N = Qhat.shape[0]
    s = (-1.0) ** np.add.outer(np.add.outer(np.arange(N), np.arange(N)), np.arange(N))
    return scipy.fft.ifftn(s * Qhat, workers=WORKERS) * N ** 3


def circular_convolution(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """sum_{l+m = k (mod N)} X_l Y_m for arrays indexed by DFT index, by FFT."""
    N = X.shape[0]
    x = scipy.fft.ifftn(X, workers=WORKERS)
    y = scipy.fft.ifftn(Y, workers=WORKERS)
    return scipy.fft.fftn(x * y, workers=WORKERS) * N ** 3


def collide_pair_fast(fi: np.ndarray, fj: np.ndarray, pr: Pair) -> np.ndarray:
    """The fast algorithm of Sec. 4 for one ordered pair and one spatial point.

    Q_hat+_k = sum_{rho,sigma} w_rho w_sigma F(k, rho, sigma)
               sum_{l+m=k} (e^{i pi rho a l.sigma/L} f_hat^i_l)(e^{-i pi rho b m.sigma/L} f_hat^j_m),
    Q_hat-_k = sum_{l+m=k} f_hat^i_l (G-(m) f_hat^j_m),
    each inner sum a convolution evaluated by FFT."""
    N = fi.shape[0]
    L = pr.L
    fhi = _coefficients_fft(fi)
    fhj = _coefficients_fft(fj)
    KX, KY, KZ = mode_grids(N)
    kabs = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    kvec = np.stack([KX, KY, KZ], axis=-1)
    Qplus = np.zeros((N, N, N), dtype=np.complex128)
    for q in range(len(pr.rho)):
        rho = pr.rho[q]
        for p in range(len(pr.wsigma)):
            if pr.alpha == 1.0:
                Fqp = pr.kernel_mode(kvec, q, p)
            else:
                Fqp = V.kernel_mode_grid(N, rho, pr.sigma[p], pr.a, pr.gamma, pr.alpha, pr.C, L)
            s = pr.sigma[p]
            ksig = KX * s[0] + KY * s[1] + KZ * s[2]
            X = np.exp(1j * np.pi * rho * pr.a * ksig / L) * fhi
            Y = np.exp(-1j * np.pi * rho * pr.b * ksig / L) * fhj
            Qplus += pr.wrho[q] * pr.wsigma[p] * Fqp * circular_convolution(X, Y)
    Gm = pr.loss(kabs)
    Qminus = circular_convolution(fhi, Gm * fhj)
    return _synthesize_fft(Qplus - Qminus).real


def _pad(X: np.ndarray, P: int) -> np.ndarray:
    """Coefficients indexed by DFT index on the N grid, placed at the same modes of a
    P grid (P >= N); every other mode zero."""
    N = X.shape[0]
    idx = np.arange(N)
    k = np.where(idx < N // 2, idx, idx - N) % P
    out = np.zeros((P, P, P), dtype=np.complex128)
    out[np.ix_(k, k, k)] = X
    return out


def _truncate(Y: np.ndarray, N: int) -> np.ndarray:
    """Modes -N/2..N/2-1 of a P-grid array, by N-grid DFT index."""
    P = Y.shape[0]
    idx = np.arange(N)
    k = np.where(idx < N // 2, idx, idx - N) % P
    return Y[np.ix_(k, k, k)]


def linear_convolution(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """sum_{l+m = k} X_l Y_m over l, m, k in [-N/2, N/2-1]^3 without wrap-around: both
    are zero-padded to a 2N grid, where l + m (in [-N, N-2]) never wraps onto a kept k."""
    N = X.shape[0]
    return _truncate(circular_convolution(_pad(X, 2 * N), _pad(Y, 2 * N)), N)


def collide_pair_dealiased(fi: np.ndarray, fj: np.ndarray, pr: Pair) -> np.ndarray:
    """Eq. (sum) read literally: the sums over l + m = k with l, m, k all in
    [-N/2, N/2-1]^3 (no wrap-around), in the quadrature form of Sec. 4 for the gain, each
    inner sum a linear convolution; the operator at a grid point is the real part of the
    synthesised series, as for the circular form."""
    N = fi.shape[0]
    L = pr.L
    fhi = _coefficients_fft(fi)
    fhj = _coefficients_fft(fj)
    KX, KY, KZ = mode_grids(N)
    kabs = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    kvec = np.stack([KX, KY, KZ], axis=-1)
    Qplus = np.zeros((N, N, N), dtype=np.complex128)
    for q in range(len(pr.rho)):
        rho = pr.rho[q]
        for p in range(len(pr.wsigma)):
            Fqp = pr.kernel_mode(kvec, q, p)
            s = pr.sigma[p]
            ksig = KX * s[0] + KY * s[1] + KZ * s[2]
            X = np.exp(1j * np.pi * rho * pr.a * ksig / L) * fhi
            Y = np.exp(-1j * np.pi * rho * pr.b * ksig / L) * fhj
            Qplus += pr.wrho[q] * pr.wsigma[p] * Fqp * linear_convolution(X, Y)
    Qminus = linear_convolution(fhi, pr.loss(kabs) * fhj)
    return _synthesize_fft(Qplus - Qminus).real


def collide_pair_fast_parts(fi: np.ndarray, fj: np.ndarray, pr: Pair):
    """Gain and loss of ``collide_pair_fast`` separately (real parts on the grid)."""
    N = fi.shape[0]
    L = pr.L
    fhi = _coefficients_fft(fi)
    fhj = _coefficients_fft(fj)
    KX, KY, KZ = mode_grids(N)
    kabs = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    Gm = pr.loss(kabs)
    Qminus = _synthesize_fft(circular_convolution(fhi, Gm * fhj)).real
    Qfull = collide_pair_fast(fi, fj, pr)
    return Qfull + Qminus, Qminus


# ---------------------------------------------------------- multi-species driver
@dataclass
class Problem:
    """A multi-species collision problem on a common grid.

    kernel[i][j] = (omega, alpha, C_ij)."""
    masses: tuple
    L: float
    N: int
    M: int
    nrho: int
    kernel: list
    sigma: np.ndarray | None = None
    wsigma: np.ndarray | None = None

    def __post_init__(self):
        if self.sigma is None:
            self.sigma, self.wsigma = Qd.design_quadrature(self.M)

    @property
    def s(self) -> int:
        return len(self.masses)

    def pair(self, i: int, j: int) -> Pair:
        omega, alpha, C = self.kernel[i][j]
        return make_pair(self.masses[i], self.masses[j], omega, C, self.L, self.nrho,
                         self.sigma, self.wsigma, alpha=alpha)


def vhs_problem(masses, omega: float, L: float, N: int, M: int, nrho: int, kn0: float = 1.0) -> Problem:
    """Problem with the dimensionless VHS kernel of eq. (NVSS) and Kn_ij^{-1} folded in."""
    s = len(masses)
    kern = [[(omega, 1.0, P.vss_prefactor(masses[i], masses[j], omega, 1.0, kn0)) for j in range(s)]
            for i in range(s)]
    return Problem(masses=tuple(masses), L=L, N=N, M=M, nrho=nrho, kernel=kern)


def collide_pairs(f: np.ndarray, prob: Problem, method: str = "fast") -> np.ndarray:
    """Q^{ij}(f^i, f^j) for every ordered pair: f [s][N][N][N] -> [s][s][N][N][N]."""
    fn = {"fast": collide_pair_fast, "direct": collide_pair_direct,
          "exact_sphere": collide_pair_exact_sphere, "dealiased": collide_pair_dealiased,
          "direct_linear": lambda a, b, pr: collide_pair_direct(a, b, pr, linear=True)}[method]
    s = prob.s
    out = np.zeros((s, s) + f.shape[1:])
    for i in range(s):
        for j in range(s):
            out[i, j] = fn(f[i], f[j], prob.pair(i, j))
    return out


def collide(f: np.ndarray, prob: Problem, method: str = "fast") -> np.ndarray:
    """The right-hand side of eq. (NMBE): Q^i = sum_j Q^{ij} (prefactors included)."""
    return collide_pairs(f, prob, method).sum(axis=1)
