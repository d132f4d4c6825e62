"""GPU parity with species-specific velocity grids: the HIP path (one single-grid part
per pair box, interpolation kernels between grids) against the oracle's reading of the
same rule, element by element.  Tolerances as in the common-grid tests: FP64 1e-12,
FP32 1e-5 relative L-inf per (node, species); pair-resolved FP32 results of inputs at
equilibrium are measured against the loss scale (the pair's own maximum is quadrature
noise there)."""
import numpy as np
import pytest

from oracle import grids as OG, moments as OM, spectral as OS
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


def _loss_scale(f, prob, Ls):
    """max_n |Q-^{ij}| per ordered pair (the loss term f^i nu^{ij} on grid i), [s][s]."""
    s = prob.s
    out = np.zeros((s, s))
    for i in range(s):
        for j in range(s):
            Lij = max(Ls[i], Ls[j])
            fi = f[i] if Ls[i] == Lij else OG.interpolate(f[i], Ls[i], Lij)
            fj = f[j] if Ls[j] == Lij else OG.interpolate(f[j], Ls[j], Lij)
            om, al, C = prob.kernel[i][j]
            pr = OS.make_pair(prob.masses[i], prob.masses[j], om, C, Lij, prob.nrho, prob.sigma, prob.wsigma)
            loss = OS.collide_pair_fast_parts(fi, fj, pr)[1]
            if Ls[i] != Lij:
                loss = OG.interpolate(loss, Lij, Ls[i])
            out[i, j] = np.abs(loss).max()
    return out


def _plan(masses, N, Ls, M, nrho, omega, precision):
    from paper_1903_03056_amd import CollisionPlan
    return CollisionPlan(masses, N, Ls, M, nrho, omega=omega, precision=precision)


def _heavy_light(N):
    masses = (1.0, 32.75)
    Ls = (6.0, 6.0 * np.sqrt(1.0 / 32.75))
    return masses, Ls


@pytest.mark.parametrize("precision,tol,N,M,nrho", [("f64", 1e-12, 16, 24, 8), ("f32", 1e-5, 24, 12, 12),
                                                 ("f32", 1e-5, 32, 6, 8)])
def test_two_species_two_grids(precision, tol, N, M, nrho):
    """m = (1, 32.75), L_i = 6 sqrt(1/m_i), hard spheres (omega = 0.5): pairs (1,1),
    (1,2), (2,1) on the wide box, (2,2) on the narrow one; summed and per pair.

    The inputs are Maxwellians at rest, so the like pairs vanish in the continuum and
    their discrete values are quadrature error of about 1e-4 of the loss term: in FP32
    the pair-resolved results are measured against the loss scale max |f^i nu^{ij}|."""
    _require_gpu()
    print(f"[case] species grids s=2 {precision} N={N} M={M}", flush=True)
    masses, Ls = _heavy_light(N)
    f = I.draw_config3_batch(np.random.default_rng(3), 3, N, Ls, masses)
    plan = _plan(masses, N, Ls, M, nrho, 0.5, precision)
    dt = torch.float64 if precision == "f64" else torch.float32
    ft = torch.tensor(f, dtype=dt, device="cuda")
    Q = plan.collide(ft).double().cpu().numpy()
    Qp = plan.collide(ft, pairs=True).double().cpu().numpy()
    prob = OS.vhs_problem(masses, 0.5, Ls[0], N, M, nrho)
    for b in range(3):
        fb = f[b].astype(np.float32).astype(np.float64) if precision == "f32" else f[b]
        refp = OG.collide_pairs(fb, prob, Ls)
        rel = _rel(Q[b], refp.sum(axis=1))
        print(f"node {b}: summed relative L-inf {rel:.3e}", flush=True)
        assert rel <= tol
        if precision == "f64":
            assert _rel(Qp[b], refp) <= tol
        else:
            err = np.abs(Qp[b] - refp).reshape(2, 2, -1).max(axis=2)
            rel_loss = err / _loss_scale(fb, prob, Ls)
            print(f"node {b}: pair errors over the loss scale {rel_loss.ravel()}", flush=True)
            assert np.all(rel_loss <= tol)


def test_three_species_three_grids_fp64():
    """m = (1, 4, 20) with L_i = 6 sqrt(1/m_i): three pair boxes (6, 3, 1.34), species 2
    and 3 carried onto wider grids and back."""
    _require_gpu()
    print("[case] species grids s=3 fp64", flush=True)
    masses = (1.0, 4.0, 20.0)
    Ls = tuple(6.0 * np.sqrt(1.0 / m) for m in masses)
    N, M, nrho = 16, 12, 6
    f = I.draw_bimaxwellian_batch(np.random.default_rng(31), 2, 3, N, Ls, masses)
    plan = _plan(masses, N, Ls, M, nrho, 0.74, "f64")
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    Q = plan.collide(ft).cpu().numpy()
    Qp = plan.collide(ft, pairs=True).cpu().numpy()
    prob = OS.vhs_problem(masses, 0.74, Ls[0], N, M, nrho)
    for b in range(2):
        refp = OG.collide_pairs(f[b], prob, Ls)
        assert _rel(Q[b], refp.sum(axis=1)) <= 1e-12
        assert _rel(Qp[b], refp) <= 1e-12


def test_species_grids_conserve_timed_and_sliced():
    """The FP64 projection on the species' own grids matches the oracle's and conserves
    to 1e-12; the timed call and a one-node workspace (slicing) give the same values bit
    for bit."""
    _require_gpu()
    print("[case] species grids conserve/timed/sliced", flush=True)
    masses, Ls = _heavy_light(16)
    N = 16
    f = I.draw_config3_batch(np.random.default_rng(5), 3, N, Ls, masses)
    plan = _plan(masses, N, Ls, 12, 6, 0.5, "f64")
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    Q = plan.collide(ft)
    Qt, stages = plan.collide_timed(ft)
    ws1 = torch.empty(plan.workspace_bytes(1), dtype=torch.uint8, device="cuda")
    Qs = plan.collide(ft, workspace=ws1)
    torch.cuda.synchronize()
    assert torch.equal(Q, Qt) and torch.equal(Q, Qs)
    assert all(t > 0 for t in stages)
    Qc = plan.conserve(Q).cpu().numpy()
    raw = Q.cpu().numpy()
    for b in range(3):
        ref = OM.conserve(raw[b], masses, Ls)
        assert np.abs(Qc[b] - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.all(OM.conservation_residual(Qc[b], masses, Ls) <= 1e-12)


def test_species_grids_reject_plain_path():
    _require_gpu()
    from paper_1903_03056_amd._lib import DgfsError
    masses, Ls = _heavy_light(16)
    plan = _plan(masses, 16, Ls, 6, 4, 0.5, "f64")
    with pytest.raises(DgfsError):
        plan.collide_plain(torch.zeros((1, 2, 16, 16, 16), dtype=torch.float64, device="cuda"))


def test_full_size_heavy_light_batch_sampled():
    """1024 nodes, N = 48, M = 24 (7-design), N_rho = 24, m = (1, 32.75) on L = (6, 1.0484),
    hard spheres, FP32, processed in slices of a 128-node workspace: the last node (in the
    final, ragged slice) against the oracle, and bit for bit equal to that node alone."""
    _require_gpu()
    print("[case] species grids full size B=1024 N=48 M=24", flush=True)
    masses, Ls = _heavy_light(48)
    N, M, nrho, B = 48, 24, 24, 1024
    f = I.draw_config3_batch(np.random.default_rng(3), B, N, Ls, masses)
    plan = _plan(masses, N, Ls, M, nrho, 0.5, "f32")
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    ws = torch.empty(plan.workspace_bytes(128), dtype=torch.uint8, device="cuda")
    Q = plan.collide(ft, workspace=ws)
    Q1 = plan.collide(ft[B - 1:].contiguous(), workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(Q[B - 1], Q1[0])
    assert torch.isfinite(Q).all()
    prob = OS.vhs_problem(masses, 0.5, Ls[0], N, M, nrho)
    fb = f[B - 1].astype(np.float32).astype(np.float64)
    ref = OG.collide(fb, prob, Ls)
    got = Q[B - 1].double().cpu().numpy()
    rel = _rel(got, ref)
    print(f"last node: relative L-inf {rel:.3e}", flush=True)
    assert rel <= 1e-5
