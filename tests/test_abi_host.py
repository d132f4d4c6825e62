"""Host-side checks of the C ABI: the library loads, exports what include/dgfs.h
declares, validates problems, and its FP64 precomputation agrees with the oracle.
No GPU is used."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import params as OP, quadrature as OQ, spectral as OS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1903_03056_amd", "libdgfs.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libdgfs.so not built")


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "dgfs.h")).read()
    return sorted(set(re.findall(r"\b(dgfs_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(LIB)
    names = _declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n


def test_binding_names_match_header():
    from paper_1903_03056_amd import _lib
    assert sorted(_lib.EXPORTED) == _declared_functions()


@pytest.mark.parametrize("mi,mj,omega,alpha,kn0", [
    (1.0, 1.0, 0.5, 1.0, 1.0), (1.0, 2.0, 0.74, 1.0, 1.0), (1.0, 32.75, 0.5, 1.0, 0.3),
    (66.3, 139.1, 0.81, 1.4, 0.04), (139.1 / 66.3, 1.0, 0.805, 1.36, 2.5), (4.0, 20.0, 1.0, 2.0, 1.0),
])
def test_pair_prefactor_matches_oracle(mi, mj, omega, alpha, kn0):
    """C_ij of eqs. (Kn), (NVSS) computed by the library equals the oracle's, and is
    symmetric in the two masses."""
    from paper_1903_03056_amd import pair_prefactor
    ref = OP.vss_prefactor(mi, mj, omega, alpha, kn0)
    assert abs(pair_prefactor(mi, mj, omega, alpha, kn0) - ref) <= 1e-15 * ref
    assert abs(pair_prefactor(mj, mi, omega, alpha, kn0) - ref) <= 1e-15 * ref


def test_pair_prefactor_rejects_bad_arguments():
    from paper_1903_03056_amd import pair_prefactor
    from paper_1903_03056_amd._lib import DGFS_EINVAL, DgfsError
    for args in [(0.0, 1.0, 0.74, 1.0, 1.0), (1.0, 1.0, 0.4, 1.0, 1.0), (1.0, 1.0, 0.74, 2.5, 1.0),
                 (1.0, 1.0, 0.74, 1.0, 0.0), (1.0, float("nan"), 0.74, 1.0, 1.0)]:
        with pytest.raises(DgfsError) as e:
            pair_prefactor(*args)
        assert e.value.status == DGFS_EINVAL


def _kern(masses, omega):
    from paper_1903_03056_amd import vhs_kernel
    return vhs_kernel(masses, omega)


def test_check_problem_accepts_and_rejects():
    from paper_1903_03056_amd import check_problem
    from paper_1903_03056_amd._lib import DGFS_EINVAL, DGFS_EUNSUPPORTED, DGFS_OK
    m = (1.0, 2.0)
    k = _kern(m, 0.74)
    assert check_problem(m, 6.0, 32, 12, 16, k) == DGFS_OK
    assert check_problem(m, 5.0, 16, 6, 8, _kern(m, 1.0), "f64") == DGFS_OK
    assert check_problem(m, 6.0, 32, 7, 16, k) == DGFS_EINVAL           # no design
    assert check_problem(m, -1.0, 32, 12, 16, k) == DGFS_EINVAL         # L
    assert check_problem(m, 6.0, 31, 12, 16, k) == DGFS_EINVAL          # odd N
    assert check_problem(m, 6.0, 32, 12, 0, k) == DGFS_EINVAL           # n_rho
    assert check_problem((1.0, -2.0), 6.0, 32, 12, 16, k) == DGFS_EINVAL
    bad = [list(r) for r in k]
    bad[0][1] = (0.74, 1.0, k[0][1][2] * 1.01)                           # asymmetric C
    assert check_problem(m, 6.0, 32, 12, 16, bad) == DGFS_EINVAL
    bad = [list(r) for r in k]
    bad[0][0] = (0.3, 1.0, 1.0)                                          # omega out of range
    assert check_problem(m, 6.0, 32, 12, 16, bad) == DGFS_EINVAL
    vss = [[(0.74, 1.4, 1.0)] * 2 for _ in range(2)]
    assert check_problem(m, 6.0, 32, 12, 16, vss) == DGFS_OK             # VSS
    vss[0][0] = (0.74, 2.5, 1.0)
    assert check_problem(m, 6.0, 32, 12, 16, vss) == DGFS_EINVAL         # alpha out of range
    assert check_problem(m, 6.0, 20, 12, 16, k) == DGFS_EUNSUPPORTED     # no kernels for N=20
    assert check_problem(m, 6.0, 32, 12, 16, k, "f64") == DGFS_OK
    assert check_problem(m, 6.0, 48, 24, 24, k) == DGFS_OK
    assert check_problem(m, 6.0, 32, 12, 16, k, L_species=(6.0, 1.0)) == DGFS_OK
    assert check_problem(m, 6.0, 32, 12, 16, k, L_species=(6.0, -1.0)) == DGFS_EINVAL
    assert check_problem(m, -1.0, 32, 12, 16, k, L_species=(6.0, 1.0)) == DGFS_OK   # L ignored


def test_plan_create_without_device_reports_error():
    """Creating a plan needs a device; on a machine without one the call fails cleanly."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_1903_03056_amd import CollisionPlan
    from paper_1903_03056_amd._lib import DgfsError
    with pytest.raises(DgfsError):
        CollisionPlan((1.0, 2.0), 16, 5.0, 6, 8, omega=1.0, precision="f64")


@pytest.mark.parametrize("M", [6, 12, 24])
def test_design_matches_oracle(M):
    from paper_1903_03056_amd import design
    assert np.allclose(design(M), OQ.spherical_design(M), atol=1e-15)


@pytest.mark.parametrize("masses,omega,L,N,nrho", [((1.0, 2.0), 0.74, 6.0, 32, 16),
                                                   ((1.0, 2.0), 1.0, 5.0, 16, 8),
                                                   ((1.0, 4.0, 20.0), 0.5, 6.0, 24, 12)])
def test_host_tables_match_oracle(masses, omega, L, N, nrho):
    """R_ij, Gauss-Legendre nodes/weights, C_ij and the loss weight G-(|m|) computed by
    the library's own FP64 host code agree with the oracle's independent routines."""
    from paper_1903_03056_amd import pair_tables
    k = _kern(masses, omega)
    s = len(masses)
    for i in range(s):
        for j in range(s):
            t = pair_tables(masses, L, N, 12, nrho, k, i, j)
            pr = OS.make_pair(masses[i], masses[j], omega, OP.vss_prefactor(masses[i], masses[j], omega), L, nrho,
                              *OQ.design_quadrature(12))
            assert t["a"] == pytest.approx(pr.a, rel=1e-15) and t["b"] == pytest.approx(pr.b, rel=1e-15)
            assert t["R"] == pytest.approx(pr.R, rel=1e-15)
            assert t["C"] == pytest.approx(pr.C, rel=1e-14)
            assert np.allclose(t["rho"], pr.rho, rtol=1e-14, atol=0)
            assert np.allclose(t["wrho"], pr.wrho, rtol=1e-13, atol=0)
            k2 = np.arange(3 * (N // 2) ** 2 + 1)
            ref = OS.loss_weight(np.sqrt(k2), pr.R, pr.gamma, pr.C, L)
            scale = np.abs(ref).max()
            assert np.abs(t["loss_by_k2"] - ref).max() <= 1e-13 * scale
            assert t["ndir"] == (6 if i == j else 12)


def test_tile_candidates_and_validation():
    from paper_1903_03056_amd import check_problem, tile_candidates
    from paper_1903_03056_amd._lib import DGFS_EUNSUPPORTED, DGFS_OK
    for N in (16, 24, 32, 48, 64):
        c32 = tile_candidates(N, "f32")
        c64 = tile_candidates(N, "f64")
        assert len(c32) >= 1 and len(c64) >= 1
        for ch, cz in c32:
            if cz == 0:   # the matrix-core gain: N = 32, two x-chunks
                assert (N, ch) == (32, 2)
                continue
            assert N % ch == 0 and N % cz == 0 and ((N // ch) * N) % 64 == 0
        assert all(cz > 0 for _, cz in c64)
    m = (1.0, 2.0)
    k = _kern(m, 0.74)
    for tile in tile_candidates(32, "f32"):
        assert check_problem(m, 6.0, 32, 12, 16, k, tile=tile) == DGFS_OK
    assert check_problem(m, 6.0, 32, 12, 16, k, tile=(3, 1)) == DGFS_EUNSUPPORTED
    # the matrix-core geometry: FP32, N = 32, VHS kernels only
    from paper_1903_03056_amd import vss_kernel as _vss
    assert tile_candidates(32, "f32")[0] == (2, 0)
    assert check_problem(m, 6.0, 32, 12, 16, _vss(m, 0.8, 1.4), tile=(2, 0)) == DGFS_EUNSUPPORTED
    assert check_problem(m, 6.0, 32, 12, 16, _vss(m, 0.8, 1.4)) == DGFS_OK
    assert check_problem(m, 6.0, 32, 12, 16, k, precision="f64", tile=(2, 0)) == DGFS_EUNSUPPORTED
    assert check_problem(m, 6.0, 16, 6, 8, k, tile=(2, 0)) == DGFS_EUNSUPPORTED
    # N = 64: VHS kernels on one or several grids; no VSS kernels, no dealiased form
    from paper_1903_03056_amd import vss_kernel
    assert check_problem(m, 12.0, 64, 6, 32, k) == DGFS_OK
    assert check_problem(m, 12.0, 64, 6, 32, k, precision="f64") == DGFS_OK
    assert check_problem(m, 12.0, 64, 6, 32, vss_kernel(m, 0.8, 1.4)) == DGFS_EUNSUPPORTED
    assert check_problem(m, 12.0, 64, 6, 32, k, dealias=True) == DGFS_EUNSUPPORTED


@pytest.mark.parametrize("N,L_from,L_to", [(8, 1.0, 2.3), (16, 1.0484, 6.0), (24, 6.0, 1.0484), (48, 2.0, 2.0)])
def test_interpolation_matrix_matches_oracle(N, L_from, L_to):
    """The library's one-dimensional map, applied along each axis, gives the oracle's
    interpolant between species grids (which it computes from the Fourier coefficients)."""
    from oracle import grids as OG
    from paper_1903_03056_amd import interpolation_matrix
    T = interpolation_matrix(N, L_from, L_to)
    f = np.random.default_rng(N).random((N, N, N))
    got = np.einsum("ai,bj,ck,ijk->abc", T, T, T, f, optimize=True)
    ref = OG.interpolate(f, L_from, L_to)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(f).max()


def test_pair_tables_use_the_pair_box_with_species_grids():
    """With species-specific grids, R_ij and G-_ij are those of the box max(L_i, L_j)."""
    from paper_1903_03056_amd import pair_tables
    masses = (1.0, 32.75)
    Ls = (6.0, 6.0 * np.sqrt(1.0 / 32.75))
    k = _kern(masses, 0.5)
    for i in range(2):
        for j in range(2):
            t = pair_tables(masses, 6.0, 16, 24, 8, k, i, j, L_species=Ls)
            Lij = max(Ls[i], Ls[j])
            assert t["R"] == pytest.approx(OP.truncation_radius(Lij, masses[i], masses[j]), rel=1e-15)
            k2 = np.arange(3 * 8 ** 2 + 1)
            ref = OS.loss_weight(np.sqrt(k2), t["R"], t["gamma"], t["C"], Lij)
            assert np.abs(t["loss_by_k2"] - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("alpha", [1.0, 1.32, 1.36, 1.4, 2.0])
def test_vss_kernel_mode_matches_oracle(alpha):
    """The library's kernel mode (Funk-Hecke series with Miller-recurrence Bessel
    functions) against the oracle's (pole-at-sigma Gauss-Jacobi integral), over modes of
    an N = 48 grid and radii up to R: within 1e-12 of F(0)."""
    from oracle import vss as OV
    from paper_1903_03056_amd import kernel_mode
    rng = np.random.default_rng(int(alpha * 100))
    sig = OQ.design_quadrature(24)[0]
    for trial in range(40):
        k = rng.integers(-24, 24, size=3).astype(float)
        sg = sig[trial % 24] if trial % 2 else rng.normal(size=3)
        sg = sg / np.linalg.norm(sg)
        rho, a, gamma, C, L = rng.uniform(0, 5.5), rng.uniform(0.02, 0.98), rng.uniform(0, 1), 0.7, 6.0
        got = kernel_mode(alpha, gamma, C, a, L, rho, k, sg)
        ref = OV.kernel_mode(k[None, :], rho, sg, a, gamma, alpha, C, L)[0]
        F0 = C * rho ** (gamma + 2) * 2 * np.pi * 2 ** alpha / alpha
        assert abs(got - ref) <= 1e-12 * F0, (k, rho, a)


def test_vss_loss_table_matches_oracle():
    """G- of a VSS pair (alpha = 1.36) from the library's tables against the oracle's."""
    from paper_1903_03056_amd import pair_tables
    m = (1.0, 2.1)
    kern = [[(0.805, 1.36, OP.vss_prefactor(m[i], m[j], 0.805, 1.36)) for j in range(2)] for i in range(2)]
    t = pair_tables(m, 6.0, 32, 12, 16, kern, 0, 1, "f64")
    R = OP.truncation_radius(6.0, m[0], m[1])
    ref = OS.loss_weight(np.sqrt(np.arange(3 * 16 ** 2 + 1)), R, 2 * (1 - 0.805), kern[0][1][2], 6.0, alpha=1.36)
    assert np.abs(t["loss_by_k2"] - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("K", [2, 3, 4, 5, 6, 7, 8])
def test_slab_gll_matches_oracle(K):
    """The library's GLL rule (bisection on P'_{K-1}) against the oracle's (numpy roots)."""
    from oracle import dg
    from paper_1903_03056_amd import slab_gll
    x, w = slab_gll(K)
    xr, wr = dg.gll(K)
    np.testing.assert_allclose(x, xr, atol=1e-14)
    np.testing.assert_allclose(w, wr, atol=1e-14)


def test_check_problem_dealias():
    from paper_1903_03056_amd import check_problem
    from paper_1903_03056_amd._lib import DGFS_EUNSUPPORTED, DGFS_OK
    m = (1.0, 2.0)
    k = _kern(m, 0.74)
    assert check_problem(m, 6.0, 16, 6, 8, k, dealias=True) == DGFS_OK
    assert check_problem(m, 6.0, 32, 12, 16, k, dealias=True) == DGFS_OK
    assert check_problem(m, 6.0, 24, 12, 12, k, dealias=True) == DGFS_OK
    assert check_problem(m, 6.0, 48, 12, 12, k, dealias=True) == DGFS_OK
    assert check_problem(m, 6.0, 64, 12, 12, k, dealias=True) == DGFS_EUNSUPPORTED    # 96 not compiled
    vss = [[(0.74, 1.4, 1.0)] * 2 for _ in range(2)]
    assert check_problem(m, 6.0, 16, 6, 8, vss, dealias=True) == DGFS_EUNSUPPORTED
    assert check_problem(m, 6.0, 16, 6, 8, k, L_species=(6.0, 3.0), dealias=True) == DGFS_EUNSUPPORTED
    assert check_problem(m, 6.0, 16, 6, 8, k, tile=(2, 1), dealias=True) == DGFS_EUNSUPPORTED
