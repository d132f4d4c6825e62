"""GPU parity with VSS kernels (alpha > 1): the sigma-dependent kernel mode, one complex
transform per direction and complex radial tables, against the oracle element by element
(FP64 1e-12, FP32 1e-5 relative L-inf per (node, species)), and at full size against the
independently checked VHS path in the limit alpha -> 1.

Kernel: the argon-krypton VSS parameters of the paper's table of collision models
(omega = 0.81 / 0.805 / 0.8, alpha = 1.4 / 1.36 / 1.32, m2/m1 = 139.1/66.3) with the
dimensionless prefactor of eq. NVSS."""
import numpy as np
import pytest

from oracle import grids as OG, params as OP, spectral as OS, stepping as OT
from synth import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MASSES = (1.0, 139.1 / 66.3)
OMEGA = ((0.81, 0.805), (0.805, 0.8))
ALPHA = ((1.4, 1.36), (1.36, 1.32))


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _kernel(masses=MASSES, omega=OMEGA, alpha=ALPHA):
    s = len(masses)
    return [[(omega[i][j], alpha[i][j], OP.vss_prefactor(masses[i], masses[j], omega[i][j], alpha[i][j]))
             for j in range(s)] for i in range(s)]


def _rel(q, ref):
    q = q.reshape(-1, q.shape[-3] * q.shape[-2] * q.shape[-1])
    ref = ref.reshape(q.shape)
    return float(np.max(np.abs(q - ref).max(axis=1) / np.abs(ref).max(axis=1)))


def _loss_scale(f, prob):
    """max_n |Q-^{ij}| per ordered pair, [s][s] (the loss term f^i nu^{ij})."""
    s, N = prob.s, f.shape[-1]
    KX, KY, KZ = OS.mode_grids(N)
    kabs = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    out = np.zeros((s, s))
    for i in range(s):
        for j in range(s):
            pr = prob.pair(i, j)
            fhi, fhj = OS._coefficients_fft(f[i]), OS._coefficients_fft(f[j])
            loss = OS._synthesize_fft(OS.circular_convolution(fhi, pr.loss(kabs) * fhj)).real
            out[i, j] = np.abs(loss).max()
    return out


def _plan(N, L, M, nrho, precision, kernel, masses=MASSES, **kw):
    from paper_1903_03056_amd import CollisionPlan
    return CollisionPlan(masses, N, L, M, nrho, kernel=kernel, precision=precision, **kw)


@pytest.mark.parametrize("M", [6, 12, 24])
def test_vss_single_point_fp64(M):
    """N = 16, N_rho = 8, L = 6, two bi-Maxwellian nodes: summed and pair-resolved
    operators within 1e-12 of the oracle (M = 24: a design that is not antipodal)."""
    _require_gpu()
    print(f"[case] vss fp64 N=16 M={M}", flush=True)
    N, L, nrho = 16, 6.0, 8
    kern = _kernel()
    plan = _plan(N, L, M, nrho, "f64", kern)
    f = I.draw_bimaxwellian_batch(np.random.default_rng(40 + M), 2, 2, N, (L, L), MASSES)
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    Q = plan.collide(ft).cpu().numpy()
    Qp = plan.collide(ft, pairs=True).cpu().numpy()
    prob = OS.Problem(masses=MASSES, L=L, N=N, M=M, nrho=nrho, kernel=kern)
    for b in range(2):
        refp = OS.collide_pairs(f[b], prob)
        rs, rp = _rel(Q[b], refp.sum(axis=1)), _rel(Qp[b], refp)
        print(f"node {b}: summed {rs:.3e}, pairs {rp:.3e}", flush=True)
        assert rs <= 1e-12 and rp <= 1e-12


@pytest.mark.parametrize("N,M,nrho", [(24, 12, 12), (32, 6, 8)])
def test_vss_fp32(N, M, nrho):
    """FP32 plans against the oracle on the FP32-rounded inputs: three nodes (the batch
    spans several tiles of the gain kernel), summed within 1e-5 relative; pair-resolved
    within 1e-5 of the pair's loss term (a like pair of near-Maxwellian data is a small
    difference of gain and loss, so its own maximum is no scale for FP32 rounding)."""
    _require_gpu()
    print(f"[case] vss fp32 N={N} M={M}", flush=True)
    L = 6.0
    kern = _kernel()
    plan = _plan(N, L, M, nrho, "f32", kern)
    f = I.draw_bimaxwellian_batch(np.random.default_rng(N), 3, 2, N, (L, L), MASSES).astype(np.float32)
    ft = torch.tensor(f, device="cuda")
    Q = plan.collide(ft).double().cpu().numpy()
    Qp = plan.collide(ft, pairs=True).double().cpu().numpy()
    prob = OS.Problem(masses=MASSES, L=L, N=N, M=M, nrho=nrho, kernel=kern)
    for b in range(3):
        fb = f[b].astype(np.float64)
        refp = OS.collide_pairs(fb, prob)
        rs = _rel(Q[b], refp.sum(axis=1))
        rp = np.abs(Qp[b] - refp).reshape(2, 2, -1).max(axis=2) / _loss_scale(fb, prob)
        print(f"node {b}: summed {rs:.3e}, pairs over the loss scale {rp.ravel()}", flush=True)
        assert rs <= 1e-5 and np.all(rp <= 1e-5)


@pytest.mark.parametrize("precision,B,tol", [("f64", 16, 1e-7), ("f32", 256, 1e-5)])
def test_vss_full_size_against_vhs_limit(precision, B, tol):
    """The 256-node N = 32, M = 12, N_rho = 16 slab shape: a VSS plan with alpha = 1 + 1e-8
    (sigma-dependent tables, one transform per direction) against the VHS plan (alpha = 1,
    one summed field per class), which differ by O(alpha - 1) in exact arithmetic; and the
    last node alone equals the same node in the batch bit for bit."""
    _require_gpu()
    print(f"[case] vss full size {precision} B={B}", flush=True)
    N, L, M, nrho = 32, 6.0, 12, 16
    masses = (1.0, 2.0)
    om = ((0.74, 0.74), (0.74, 0.74))
    near = ((1.0 + 1e-8,) * 2,) * 2
    vss = _plan(N, L, M, nrho, precision, _kernel(masses, om, near), masses=masses)
    vhs = _plan(N, L, M, nrho, precision, _kernel(masses, om, ((1.0,) * 2,) * 2), masses=masses)
    dt = torch.float64 if precision == "f64" else torch.float32
    f = I.draw_bimaxwellian_batch(np.random.default_rng(2), B, 2, N, (L, L), masses, noise=1e-2)
    ft = torch.tensor(f, dtype=dt, device="cuda")
    Qv = vss.collide(ft)
    Qh = vhs.collide(ft)
    Q1 = vss.collide(ft[B - 1:].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(Qv[B - 1], Q1[0])
    rel = max(_rel(Qv[b].double().cpu().numpy(), Qh[b].double().cpu().numpy()) for b in range(B))
    print(f"max relative L-inf VSS(alpha=1+1e-8) vs VHS: {rel:.3e}", flush=True)
    assert rel <= tol


def test_vss_species_grids_fp64():
    """VSS kernels on species-specific grids (m = (1, 2.098) on L = (6, 4.14)): the pair
    boxes, interpolation and complex tables together, within 1e-12 of the oracle."""
    _require_gpu()
    print("[case] vss species grids fp64", flush=True)
    N, M, nrho = 16, 12, 6
    Ls = tuple(6.0 * np.sqrt(1.0 / m) for m in MASSES)
    kern = _kernel()
    plan = _plan(N, Ls, M, nrho, "f64", kern)
    f = I.draw_bimaxwellian_batch(np.random.default_rng(9), 1, 2, N, Ls, MASSES)
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    Q = plan.collide(ft).cpu().numpy()
    prob = OS.Problem(masses=MASSES, L=Ls[0], N=N, M=M, nrho=nrho, kernel=kern)
    rel = _rel(Q[0], OG.collide(f[0], prob, Ls))
    print(f"relative L-inf {rel:.3e}", flush=True)
    assert rel <= 1e-12


def test_vss_relax_fp64():
    """Two SSP-RK2 steps of the projected VSS operator against the oracle's stepping."""
    _require_gpu()
    print("[case] vss relax fp64", flush=True)
    N, L, M, nrho = 16, 6.0, 6, 8
    kern = _kernel()
    plan = _plan(N, L, M, nrho, "f64", kern)
    f = I.draw_bimaxwellian_batch(np.random.default_rng(12), 1, 2, N, (L, L), MASSES)
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    plan.relax(ft, 0.05, 2)
    prob = OS.Problem(masses=MASSES, L=L, N=N, M=M, nrho=nrho, kernel=kern)
    ref = OT.ssprk2(f[0], OT.collision_rhs(prob), 0.05, 2)
    got = ft[0].cpu().numpy()
    rel = max(float(np.abs(got[i] - ref[i]).max() / np.abs(ref[i]).max()) for i in range(2))
    print(f"state relative L-inf {rel:.3e}", flush=True)
    assert rel <= 1e-12


def test_vss_plain_path_is_rejected():
    _require_gpu()
    from paper_1903_03056_amd._lib import DgfsError
    plan = _plan(16, 6.0, 6, 4, "f64", _kernel())
    with pytest.raises(DgfsError):
        plan.collide_plain(torch.zeros((1, 2, 16, 16, 16), dtype=torch.float64, device="cuda"))


def test_vss_three_species_pairs_fp64():
    """Three species (m = 1, 2.098, 4) with VSS kernels, N = 16, M = 12, N_rho = 6, FP64:
    the summed operator (three slots) and the pair-resolved one (nine slots, the radial
    kernel's one-slot-per-thread form) within 1e-12 of the oracle."""
    _require_gpu()
    print("[case] vss three species pairs fp64", flush=True)
    masses = (1.0, 139.1 / 66.3, 4.0)
    om = ((0.81, 0.805, 0.79), (0.805, 0.8, 0.78), (0.79, 0.78, 0.77))
    al = ((1.4, 1.36, 1.3), (1.36, 1.32, 1.25), (1.3, 1.25, 1.2))
    kern = _kernel(masses, om, al)
    N, L, M, nrho = 16, 6.0, 12, 6
    plan = _plan(N, L, M, nrho, "f64", kern, masses=masses)
    f = I.draw_bimaxwellian_batch(np.random.default_rng(77), 2, 3, N, (L,) * 3, masses)
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    Q = plan.collide(ft).cpu().numpy()
    Qp = plan.collide(ft, pairs=True).cpu().numpy()
    prob = OS.Problem(masses=masses, L=L, N=N, M=M, nrho=nrho, kernel=kern)
    for b in range(2):
        refp = OS.collide_pairs(f[b], prob)
        rs, rp = _rel(Q[b], refp.sum(axis=1)), _rel(Qp[b], refp)
        print(f"node {b}: summed {rs:.3e}, pairs {rp:.3e}", flush=True)
        assert rs <= 1e-12 and rp <= 1e-12
