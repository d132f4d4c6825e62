"""Seeded synthetic distribution functions for the collision-operator workloads.

Every workload draws with ``numpy.random.default_rng(seed)`` (PCG64) in the fixed
order node -> species -> Maxwellian component -> parameter; additive noise, when a
workload has it, is drawn afterwards for the whole batch at once.

The velocity grid of a species with half-width L is v_n = -L + n*2L/N, n = 0..N-1,
in every dimension, so v_{N/2} = 0 is the centre line (Sec. 6.1 slices the
distribution along f(:, N/2, N/2)).  Arrays are laid out [batch][species][N][N][N]
with the last (z) index fastest.

The Maxwellian is the nondimensional one of Sec. 3:
    M(v) = n (m / (pi T))^{3/2} exp(-m |v - u|^2 / T).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "velocity_grid",
    "maxwellian",
    "CONFIGS",
    "config",
    "draw_bimaxwellian_batch",
    "draw_config3_batch",
    "draw_uneven_groups",
    "draw_request_state",
]


def velocity_grid(N: int, L: float) -> np.ndarray:
    """1-D grid points v_n = -L + n * 2L/N (float64)."""
    return -L + np.arange(N, dtype=np.float64) * (2.0 * L / N)


def maxwellian(N: int, L: float, m: float, n: float, u, T: float) -> np.ndarray:
    """Nondimensional Maxwellian of Sec. 3 sampled on the N^3 grid of half-width L."""
    v = velocity_grid(N, L)
    u = np.asarray(u, dtype=np.float64)
    ex = np.exp(-m * (v - u[0]) ** 2 / T)
    ey = np.exp(-m * (v - u[1]) ** 2 / T)
    ez = np.exp(-m * (v - u[2]) ** 2 / T)
    return n * (m / (np.pi * T)) ** 1.5 * ex[:, None, None] * ey[None, :, None] * ez[None, None, :]


# Workload table.  Values not stated by the workload descriptions are filled as
# follows: L=6 where a workload gives none (taken from the N=32 slab workload),
# omega=0.74 for the uneven-batch and serving workloads, N_rho = N/2 there.
CONFIGS = {
    1: dict(
        name="single point, 2 species, N=16 (Maxwell molecules)",
        s=2, masses=(1.0, 2.0), omega=1.0, alpha=1.0, N=16, L=5.0, M=6, nrho=8,
        batch=1, seed=1, noise=0.0, precision="f64",
    ),
    2: dict(
        name="1D DG slab 64 elements x 4 nodes, 2 species, N=32",
        s=2, masses=(1.0, 2.0), omega=0.74, alpha=1.0, N=32, L=6.0, M=12, nrho=16,
        batch=256, seed=2, noise=1e-2, precision="f32",
    ),
    3: dict(
        name="large mass ratio, 1024 points, N=48, species-specific grids",
        s=2, masses=(1.0, 32.75), omega=0.5, alpha=1.0, N=48, L=6.0, M=24, nrho=24,
        batch=1024, seed=3, noise=0.0, precision="f32",
    ),
    4: dict(
        name="uneven batch, 3 species, N in {24, 32, 48}",
        s=3, masses=(1.0, 2.0, 4.0), omega=0.74, alpha=1.0, L=6.0, M=12,
        groups=((24, 512), (32, 256), (48, 64)), seed=4, noise=0.0, precision="f32",
    ),
}


def config(idx: int) -> dict:
    """A copy of the workload description ``idx``."""
    return dict(CONFIGS[idx])


def draw_bimaxwellian_batch(rng: np.random.Generator, batch: int, s: int, N: int, L,
                            masses, noise: float = 0.0) -> np.ndarray:
    """Per node and species, the sum of two Maxwellians with
    density ~ U(0.5, 1.5), bulk velocity ~ U(-0.5, 0.5)^3, temperature ~ U(0.5, 1.5).

    ``L`` is a scalar or one half-width per species.  With ``noise`` > 0 every grid
    value then receives noise * max(f) * U(-1, 1) (max over that node's species
    field) and the result is clipped at zero.
    """
    Ls = np.broadcast_to(np.asarray(L, dtype=np.float64), (s,))
    f = np.empty((batch, s, N, N, N), dtype=np.float64)
    for b in range(batch):
        for i in range(s):
            acc = np.zeros((N, N, N))
            for _c in range(2):
                n = rng.uniform(0.5, 1.5)
                u = rng.uniform(-0.5, 0.5, size=3)
                T = rng.uniform(0.5, 1.5)
                acc += maxwellian(N, Ls[i], masses[i], n, u, T)
            f[b, i] = acc
    if noise > 0.0:
        peak = f.reshape(batch, s, -1).max(axis=2)[:, :, None, None, None]
        f = f + noise * peak * rng.uniform(-1.0, 1.0, size=f.shape)
        np.maximum(f, 0.0, out=f)
    return f


def draw_config3_batch(rng: np.random.Generator, batch: int, N: int, L, masses) -> np.ndarray:
    """Two species at rest: density ~ U(0.5, 1.5) each, T_1 = 1 and T_2 = r T_1 with
    r ~ U(0.8, 1.25) per node.  ``L`` holds the half-width of each species' grid."""
    Ls = np.asarray(L, dtype=np.float64)
    f = np.empty((batch, 2, N, N, N), dtype=np.float64)
    for b in range(batch):
        n1 = rng.uniform(0.5, 1.5)
        n2 = rng.uniform(0.5, 1.5)
        r = rng.uniform(0.8, 1.25)
        f[b, 0] = maxwellian(N, Ls[0], masses[0], n1, (0.0, 0.0, 0.0), 1.0)
        f[b, 1] = maxwellian(N, Ls[1], masses[1], n2, (0.0, 0.0, 0.0), r)
    return f


def draw_uneven_groups(seed: int, groups, s: int, L: float, masses) -> list:
    """The uneven-N workload: one generator seeded with ``seed`` draws the classes in
    the order given, ``groups`` = ((N, batch), ...), each by
    ``draw_bimaxwellian_batch`` (float64 arrays [batch][s][N][N][N])."""
    rng = np.random.default_rng(seed)
    return [draw_bimaxwellian_batch(rng, B, s, N, L, masses) for N, B in groups]


def draw_request_state(seed: int, rid: int, masses, N: int, L: float) -> np.ndarray:
    """Initial two-Maxwellian state of one serving request, [s][N][N][N] float64, from a
    generator seeded with the pair (seed, request id)."""
    rng = np.random.default_rng([seed, rid])
    return draw_bimaxwellian_batch(rng, 1, len(masses), N, L, masses)[0]
