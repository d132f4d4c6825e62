"""Pins of the time-stepping oracle: the SSP-RK2 amplification factor on the linear test
equation, second-order convergence on an equation with a closed-form solution, and the
Krook-Wu solution of Sec. 6.1 advanced in time with the collision operator."""
import json
import os

import numpy as np
import pytest

from oracle import bkw, spectral as S, stepping as T

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_linear_amplification_factors():
    """df/dt = lam f: one SSP-RK2 step multiplies by 1 + z + z^2/2 (z = lam dt), one
    Euler step by 1 + z (complex lam exercises both stages)."""
    lam = -1.3 + 0.7j
    dt = 0.1
    z = lam * dt
    f0 = np.array([1.0 + 0.5j, -2.0 + 0.0j])
    rhs = lambda f: lam * f
    np.testing.assert_allclose(T.ssprk2(f0, rhs, dt, 1), (1 + z + z * z / 2) * f0, rtol=1e-15)
    np.testing.assert_allclose(T.euler(f0, rhs, dt, 1), (1 + z) * f0, rtol=1e-15)


def test_second_order_convergence():
    """df/dt = -f^2 with f(t) = f0 / (1 + f0 t): halving dt divides the SSP-RK2 error by
    about 4 and the Euler error by about 2."""
    f0, t1 = np.array([1.5]), 1.0
    exact = f0 / (1 + f0 * t1)
    rhs = lambda f: -f * f
    e_rk = [abs(T.ssprk2(f0, rhs, t1 / n, n) - exact)[0] for n in (20, 40, 80)]
    e_eu = [abs(T.euler(f0, rhs, t1 / n, n) - exact)[0] for n in (20, 40, 80)]
    for a, b in zip(e_rk, e_rk[1:]):
        assert 3.6 < a / b < 4.4
    for a, b in zip(e_eu, e_eu[1:]):
        assert 1.8 < a / b < 2.2


def _bkw_problem(kw, N, nrho, L=12.0, M=6):
    kern = [[(1.0, 1.0, kw.kernel_constant(i + 1, j + 1)) for j in range(2)] for i in range(2)]
    return S.Problem(masses=kw.m, L=L, N=N, M=M, nrho=nrho, kernel=kern)


@pytest.mark.parametrize("ratio", [1.0, 2.0])
def test_krook_wu_in_time(ratio):
    """The Krook-Wu solution (Sec. 6.1; m1/m2 = ratio, m2 = 1, L = 12, M = 6) advanced
    from t = 5.5 to t = 6.0 by SSP-RK2 (dt = 0.1) with the projected operator: at N = 32
    the error is within 2 x (the larger Table 1 df/dt error at N = 32, N_rho = 16) x the
    elapsed time, and the N = 32 result is closer to the exact solution than the N = 16
    one."""
    kw = bkw.KrookWu(ratio, 1.0)
    t0, t1, steps = 5.5, 6.0, 5
    errs = {}
    for N, nrho in ((16, 8), (32, 16)):
        f0, _ = kw.on_grid(N, 12.0, t0)
        fe, _ = kw.on_grid(N, 12.0, t1)
        f = T.ssprk2(f0, T.collision_rhs(_bkw_problem(kw, N, nrho)), (t1 - t0) / steps, steps)
        errs[N] = max(np.abs(f[i] - fe[i]).max() for i in range(2))
    with open(os.path.join(GOLD, "krook_wu_table1.json")) as fh:
        row = next(r for r in json.load(fh)["rows"] if r["N"] == 32 and r["nrho"] == 16)
    table1_n32 = max(row[str(int(ratio))])
    assert errs[32] < 2 * table1_n32 * (t1 - t0)
    assert errs[32] < errs[16]
