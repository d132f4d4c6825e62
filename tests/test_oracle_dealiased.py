"""Pins of the dealiased (linear-convolution) reading of eq. (sum): the padded FFT form
equals the explicit O(N^6) sum restricted to l + m in range, it equals the circular form
when the spectra are supported in |k| < N/4 (nothing can wrap), and the padded linear
convolution equals a brute-force double loop."""
import numpy as np
import pytest

from oracle import quadrature as Qd, spectral as S


def test_linear_convolution_brute_force():
    rng = np.random.default_rng(0)
    N = 4
    X = rng.normal(size=(N,) * 3) + 1j * rng.normal(size=(N,) * 3)
    Y = rng.normal(size=(N,) * 3) + 1j * rng.normal(size=(N,) * 3)
    k = S.signed_modes(N)
    ref = np.zeros((N,) * 3, dtype=complex)
    pos = {int(m): i for i, m in enumerate(k)}
    for a in range(N):
        for b in range(N):
            for c in range(N):
                for d in range(N):
                    for e in range(N):
                        for f in range(N):
                            t = (k[a] + k[d], k[b] + k[e], k[c] + k[f])
                            if all(-N // 2 <= x <= N // 2 - 1 for x in t):
                                ref[pos[t[0]], pos[t[1]], pos[t[2]]] += X[a, b, c] * Y[d, e, f]
    np.testing.assert_allclose(S.linear_convolution(X, Y), ref, atol=1e-12)


@pytest.mark.parametrize("alpha", [1.0, 1.36])
def test_dealiased_equals_direct_linear_sum(alpha):
    """N = 4: the zero-padded fast form equals eq. (sum) as an explicit double loop over
    in-range l + m (VHS and VSS kernels)."""
    rng = np.random.default_rng(1)
    N, L = 4, 4.0
    sig, ws = Qd.design_quadrature(6)
    pr = S.make_pair(1.0, 2.0, 0.74, 0.9, L, 3, sig, ws, alpha=alpha)
    fi, fj = rng.random((N,) * 3), rng.random((N,) * 3)
    fast = S.collide_pair_dealiased(fi, fj, pr)
    direct = S.collide_pair_direct(fi, fj, pr, linear=True)
    np.testing.assert_allclose(fast, direct, rtol=0, atol=1e-12 * np.abs(direct).max())
    # and it is not the circular form
    assert np.abs(S.collide_pair_fast(fi, fj, pr) - fast).max() > 1e-6 * np.abs(fast).max()


def test_dealiased_equals_circular_without_high_modes():
    """N = 16 with both spectra supported in |k| < N/4: no l + m leaves the kept range,
    so the dealiased and circular forms agree to rounding."""
    rng = np.random.default_rng(2)
    N, L = 16, 5.0
    k = S.signed_modes(N)
    low = (np.abs(k)[:, None, None] < N // 4) & (np.abs(k)[None, :, None] < N // 4) & (np.abs(k)[None, None, :] < N // 4)

    def field():
        c = np.where(low, rng.normal(size=(N,) * 3) + 1j * rng.normal(size=(N,) * 3), 0)
        c = 0.5 * (c + np.conj(c[np.ix_(*(((-np.arange(N)) % N),) * 3)]))    # Hermitian: a real field
        return S._synthesize_fft(c).real
    fi, fj = field(), field()
    sig, ws = Qd.design_quadrature(6)
    pr = S.make_pair(1.0, 2.0, 0.74, 0.9, L, 4, sig, ws)
    a = S.collide_pair_dealiased(fi, fj, pr)
    b = S.collide_pair_fast(fi, fj, pr)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * np.abs(b).max())
