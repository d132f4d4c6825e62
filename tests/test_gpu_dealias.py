"""GPU parity of the dealiased form of eq. (sum) (l + m = k without wrap-around, spectra
zero-padded to 3N/2 on the device: 24, 36, 48, 72 for N = 16, 24, 32, 48) against the
oracle's linear-convolution reading:
FP64 within 1e-12, FP32 within 1e-5 relative L-inf per (node, species)."""
import numpy as np
import pytest

from oracle import moments as OM, spectral as OS
from synth import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rel(q, ref):
    q = q.reshape(-1, q.shape[-3] * q.shape[-2] * q.shape[-1])
    ref = ref.reshape(q.shape)
    return float(np.max(np.abs(q - ref).max(axis=1) / np.abs(ref).max(axis=1)))


def _plan(masses, N, L, M, nrho, precision):
    from paper_1903_03056_amd import CollisionPlan
    return CollisionPlan(masses, N, L, M, nrho, omega=0.74, precision=precision, dealias=True)


@pytest.mark.parametrize("M", [6, 12])
def test_dealiased_fp64_N16(M):
    """Two nodes, summed and pair-resolved, against the oracle's linear convolution; the
    circular form differs from both by far more than the tolerance."""
    _require_gpu()
    print(f"[case] dealiased fp64 N=16 M={M}", flush=True)
    masses, N, L, nrho = (1.0, 2.0), 16, 5.0, 8
    plan = _plan(masses, N, L, M, nrho, "f64")
    f = I.draw_bimaxwellian_batch(np.random.default_rng(60 + M), 2, 2, N, (L, L), masses, noise=1e-2)
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    Q = plan.collide(ft).cpu().numpy()
    Qp = plan.collide(ft, pairs=True).cpu().numpy()
    prob = OS.vhs_problem(masses, 0.74, L, N, M, nrho)
    for b in range(2):
        refp = OS.collide_pairs(f[b], prob, method="dealiased")
        circ = OS.collide(f[b], prob)
        rs, rp = _rel(Q[b], refp.sum(axis=1)), _rel(Qp[b], refp)
        gap = _rel(circ, refp.sum(axis=1))
        print(f"node {b}: summed {rs:.3e}, pairs {rp:.3e}; circular vs linear {gap:.3e}", flush=True)
        assert rs <= 1e-12 and rp <= 1e-12
        assert gap > 1e-8


def test_dealiased_fp32_full_size_sampled():
    """The 256-node N = 32, M = 12, N_rho = 16 slab shape in FP32: the last node against
    the oracle, and equal bit for bit to that node alone; the FP64 conservation projection
    of the result conserves to 1e-12."""
    _require_gpu()
    print("[case] dealiased fp32 full size", flush=True)
    masses, N, L, M, nrho, B = (1.0, 2.0), 32, 6.0, 12, 16, 256
    plan = _plan(masses, N, L, M, nrho, "f32")
    f = I.draw_bimaxwellian_batch(np.random.default_rng(2), B, 2, N, (L, L), masses, noise=1e-2).astype(np.float32)
    ft = torch.tensor(f, device="cuda")
    Q = plan.collide(ft)
    Q1 = plan.collide(ft[B - 1:].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(Q[B - 1], Q1[0])
    prob = OS.vhs_problem(masses, 0.74, L, N, M, nrho)
    ref = OS.collide(f[B - 1].astype(np.float64), prob, method="dealiased")
    rel = _rel(Q[B - 1].double().cpu().numpy(), ref)
    print(f"last node: relative L-inf {rel:.3e}", flush=True)
    assert rel <= 1e-5
    Qc = plan.conserve(Q[:2]).cpu().numpy()
    for b in range(2):
        assert np.all(OM.conservation_residual(Qc[b], masses, (L, L)) <= 1e-12)


@pytest.mark.parametrize("N", [24, 48])
@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_dealiased_N24_N48(N, precision, tol):
    """The padded grids of length 36 and 72 (radix 3 twice): one noisy node, M = 6,
    N_rho = 4, summed and pair-resolved against the oracle's linear convolution (which pads
    to 2N)."""
    _require_gpu()
    print(f"[case] dealiased {precision} N={N}", flush=True)
    masses, L, M, nrho = (1.0, 2.0), 6.0, 6, 4
    plan = _plan(masses, N, L, M, nrho, precision)
    f = I.draw_bimaxwellian_batch(np.random.default_rng(70 + N), 1, 2, N, (L, L), masses, noise=1e-2)
    if precision == "f32":
        f = f.astype(np.float32).astype(np.float64)
    ft = torch.tensor(f, dtype=plan.dtype, device="cuda")
    Q = plan.collide(ft).double().cpu().numpy()
    Qp = plan.collide(ft, pairs=True).double().cpu().numpy()
    prob = OS.vhs_problem(masses, 0.74, L, N, M, nrho)
    refp = OS.collide_pairs(f[0], prob, method="dealiased")
    rs, rp = _rel(Q[0], refp.sum(axis=1)), _rel(Qp[0], refp)
    print(f"summed {rs:.3e}, pairs {rp:.3e}", flush=True)
    assert rs <= tol and rp <= tol


def test_dealiased_rejections():
    _require_gpu()
    from paper_1903_03056_amd._lib import DgfsError
    plan = _plan((1.0, 2.0), 16, 5.0, 6, 4, "f64")
    with pytest.raises(DgfsError):
        plan.collide_plain(torch.zeros((1, 2, 16, 16, 16), dtype=torch.float64, device="cuda"))
    with pytest.raises(DgfsError):
        _plan((1.0, 2.0), 64, 5.0, 6, 4, "f64")
