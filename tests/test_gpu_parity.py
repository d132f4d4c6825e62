"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element by
element on the same seeded inputs.

Tolerances: FP64 plans agree with the oracle to 1e-12 relative L-inf; FP32 plans to
1e-5 relative L-inf (the accuracy target of the FP32 path), where
    rel = max over (node, species) of max_n |Q_gpu - Q_ref| / max_n |Q_ref|.
"""
import numpy as np
import pytest

from oracle import moments as OM, spectral as OS
from synth import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _plan(masses, N, L, M, nrho, omega, precision):
    from paper_1903_03056_amd import CollisionPlan
    return CollisionPlan(masses, N, L, M, nrho, omega=omega, precision=precision)


def _oracle_problem(masses, omega, L, N, M, nrho):
    return OS.vhs_problem(masses, omega, L, N, M, nrho)


def _rel(q, ref):
    """max over leading index pairs of max|q - ref| / max|ref|."""
    q = q.reshape(-1, q.shape[-3] * q.shape[-2] * q.shape[-1])
    ref = ref.reshape(q.shape)
    return float(np.max(np.abs(q - ref).max(axis=1) / np.abs(ref).max(axis=1)))


def _run(plan, f64, pairs=False, **kw):
    dt = torch.float64 if plan.precision == 1 else torch.float32
    f = torch.tensor(f64, dtype=dt, device="cuda")
    Q = plan.collide(f, pairs=pairs, **kw)
    torch.cuda.synchronize()
    return Q.double().cpu().numpy()


# ------------------------------------------------------------- small N, FP64
@pytest.mark.parametrize("omega", [1.0, 0.5])
def test_single_point_N16_fp64(omega):
    """Single point, 2 species, m = (1, 2), N = 16, L = 5, M = 6, N_rho = 8 (FP64)."""
    _require_gpu()
    print(f"[case] N=16 fp64 omega={omega}", flush=True)
    rng = np.random.default_rng(1)
    f = I.draw_bimaxwellian_batch(rng, 1, 2, 16, 5.0, (1.0, 2.0))
    Q = _run(_plan((1.0, 2.0), 16, 5.0, 6, 8, omega, "f64"), f)
    ref = OS.collide(f[0], _oracle_problem((1.0, 2.0), omega, 5.0, 16, 6, 8))
    assert _rel(Q[0], ref) <= 1e-12


def test_single_point_N16_fp32():
    _require_gpu()
    print("[case] N=16 fp32", flush=True)
    rng = np.random.default_rng(1)
    f = I.draw_bimaxwellian_batch(rng, 1, 2, 16, 5.0, (1.0, 2.0))
    Q = _run(_plan((1.0, 2.0), 16, 5.0, 6, 8, 1.0, "f32"), f.astype(np.float32).astype(np.float64))
    ref = OS.collide(f[0].astype(np.float32).astype(np.float64), _oracle_problem((1.0, 2.0), 1.0, 5.0, 16, 6, 8))
    assert _rel(Q[0], ref) <= 1e-5


def test_pairs_mode_fp64():
    """Per ordered pair Q^{ij} (the cross classes share S_q with an antipodal design)."""
    _require_gpu()
    print("[case] pairs N=16 fp64 M=12", flush=True)
    rng = np.random.default_rng(5)
    masses = (1.0, 2.0)
    f = I.draw_bimaxwellian_batch(rng, 2, 2, 16, 5.0, masses, noise=1e-2)
    Q = _run(_plan(masses, 16, 5.0, 12, 8, 0.74, "f64"), f, pairs=True)
    prob = _oracle_problem(masses, 0.74, 5.0, 16, 12, 8)
    for b in range(2):
        ref = OS.collide_pairs(f[b], prob)
        assert _rel(Q[b], ref) <= 1e-12


def test_non_antipodal_design_fp64():
    """M = 24 (chiral 7-design): every ordered pair is its own class."""
    _require_gpu()
    print("[case] N=16 fp64 M=24", flush=True)
    rng = np.random.default_rng(7)
    masses = (1.0, 4.0)
    f = I.draw_bimaxwellian_batch(rng, 1, 2, 16, 6.0, masses)
    Q = _run(_plan(masses, 16, 6.0, 24, 6, 0.5, "f64"), f, pairs=True)
    ref = OS.collide_pairs(f[0], _oracle_problem(masses, 0.5, 6.0, 16, 24, 6))
    assert _rel(Q[0], ref) <= 1e-12


def test_one_species_and_three_species_fp64():
    _require_gpu()
    print("[case] s=1 and s=3 N=16 fp64", flush=True)
    rng = np.random.default_rng(9)
    f1 = I.draw_bimaxwellian_batch(rng, 1, 1, 16, 5.0, (1.0,))
    Q1 = _run(_plan((1.0,), 16, 5.0, 6, 8, 0.74, "f64"), f1)
    assert _rel(Q1[0], OS.collide(f1[0], _oracle_problem((1.0,), 0.74, 5.0, 16, 6, 8))) <= 1e-12
    masses = (1.0, 2.0, 4.0)
    f3 = I.draw_bimaxwellian_batch(rng, 1, 3, 16, 6.0, masses)
    Q3 = _run(_plan(masses, 16, 6.0, 12, 8, 0.74, "f64"), f3)
    assert _rel(Q3[0], OS.collide(f3[0], _oracle_problem(masses, 0.74, 6.0, 16, 12, 8))) <= 1e-12


# ---------------------------------------------------------------- N = 24
@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_three_species_N24(precision, tol):
    """3 species m = (1, 2, 4), N = 24, M = 12, N_rho = 12 (one node)."""
    _require_gpu()
    print(f"[case] N=24 s=3 {precision}", flush=True)
    rng = np.random.default_rng(4)
    masses = (1.0, 2.0, 4.0)
    f = I.draw_bimaxwellian_batch(rng, 1, 3, 24, 6.0, masses)
    if precision == "f32":
        f = f.astype(np.float32).astype(np.float64)
    Q = _run(_plan(masses, 24, 6.0, 12, 12, 0.74, precision), f)
    ref = OS.collide(f[0], _oracle_problem(masses, 0.74, 6.0, 24, 12, 12))
    assert _rel(Q[0], ref) <= tol


# ---------------------------------------------------------------- N = 48
@pytest.mark.parametrize("precision,tol", [("f32", 1e-5), ("f64", 1e-12)])
def test_two_species_N48(precision, tol):
    """N = 48 (the largest grid), masses (1, 2), M = 6, N_rho = 8, two nodes."""
    _require_gpu()
    print(f"[case] N=48 {precision}", flush=True)
    rng = np.random.default_rng(48)
    masses = (1.0, 2.0)
    f = I.draw_bimaxwellian_batch(rng, 2, 2, 48, 6.0, masses, noise=1e-2)
    if precision == "f32":
        f = f.astype(np.float32).astype(np.float64)
    Q = _run(_plan(masses, 48, 6.0, 6, 8, 0.74, precision), f)
    prob = _oracle_problem(masses, 0.74, 6.0, 48, 6, 8)
    for b in range(2):
        assert _rel(Q[b], OS.collide(f[b], prob)) <= tol, b


def test_two_species_N32_fp64():
    _require_gpu()
    print("[case] N=32 fp64", flush=True)
    rng = np.random.default_rng(32)
    masses = (1.0, 2.0)
    f = I.draw_bimaxwellian_batch(rng, 1, 2, 32, 6.0, masses, noise=1e-2)
    Q = _run(_plan(masses, 32, 6.0, 12, 8, 0.74, "f64"), f)
    assert _rel(Q[0], OS.collide(f[0], _oracle_problem(masses, 0.74, 6.0, 32, 12, 8))) <= 1e-12


# ------------------------------------------------- N = 32 slab workload (FP32)
def _slab_inputs(batch, seed=2):
    rng = np.random.default_rng(seed)
    f = I.draw_bimaxwellian_batch(rng, batch, 2, 32, 6.0, (1.0, 2.0), noise=1e-2)
    return f.astype(np.float32).astype(np.float64)


def test_slab_N32_ragged_batch():
    """N = 32, M = 12, N_rho = 16, omega = 0.74, bi-Maxwellian + 1e-2 noise; a batch of
    9 nodes (not a multiple of the 8 XCDs) checked node by node against the oracle."""
    _require_gpu()
    print("[case] N=32 fp32 batch 9", flush=True)
    f = _slab_inputs(9)
    Q = _run(_plan((1.0, 2.0), 32, 6.0, 12, 16, 0.74, "f32"), f)
    prob = _oracle_problem((1.0, 2.0), 0.74, 6.0, 32, 12, 16)
    for b in (0, 4, 8):
        assert _rel(Q[b], OS.collide(f[b], prob)) <= 1e-5, b


def test_slab_N32_full_batch_sampled():
    """The full 256-node workload in the launch configuration the benchmark times;
    sampled nodes against the oracle, and each node equal bit for bit to the same
    node computed alone (nodes are independent)."""
    _require_gpu()
    print("[case] N=32 fp32 batch 256", flush=True)
    f = _slab_inputs(256)
    plan = _plan((1.0, 2.0), 32, 6.0, 12, 16, 0.74, "f32")
    Q = _run(plan, f)
    prob = _oracle_problem((1.0, 2.0), 0.74, 6.0, 32, 12, 16)
    for b in (0, 131, 255):
        assert _rel(Q[b], OS.collide(f[b], prob)) <= 1e-5, b
        alone = _run(plan, f[b:b + 1])
        assert np.array_equal(alone[0], Q[b]), b


def test_workspace_slicing_is_bitwise_identical():
    _require_gpu()
    print("[case] N=16 slicing", flush=True)
    rng = np.random.default_rng(11)
    f = I.draw_bimaxwellian_batch(rng, 7, 2, 16, 5.0, (1.0, 2.0), noise=1e-2)
    plan = _plan((1.0, 2.0), 16, 5.0, 12, 8, 0.74, "f32")
    full = _run(plan, f)
    small = torch.empty(plan.workspace_bytes(3), dtype=torch.uint8, device="cuda")
    sliced = _run(plan, f, workspace=small)
    assert np.array_equal(full, sliced)
    again = _run(plan, f)
    assert np.array_equal(full, again)   # deterministic


def test_empty_batch_and_errors():
    _require_gpu()
    print("[case] edge cases", flush=True)
    from paper_1903_03056_amd._lib import DgfsError
    plan = _plan((1.0, 2.0), 16, 5.0, 6, 8, 1.0, "f64")
    f = torch.zeros((0, 2, 16, 16, 16), dtype=torch.float64, device="cuda")
    assert plan.collide(f).shape == (0, 2, 16, 16, 16)
    with pytest.raises(TypeError):
        plan.collide(torch.zeros((1, 2, 16, 16, 16), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        plan.collide(torch.zeros((1, 3, 16, 16, 16), dtype=torch.float64, device="cuda"))
    tiny = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(DgfsError):
        plan.collide(torch.zeros((1, 2, 16, 16, 16), dtype=torch.float64, device="cuda"), workspace=tiny)
    # zero input gives exactly zero
    z = plan.collide(torch.zeros((2, 2, 16, 16, 16), dtype=torch.float64, device="cuda"))
    assert float(z.abs().max()) == 0.0


# -------------------------------------------- tiles, uneven groups, graphs
@pytest.mark.parametrize("N,M,nrho", [(32, 12, 16), (48, 6, 8), (24, 12, 12), (16, 6, 8)])
def test_every_tile_geometry_matches_oracle(N, M, nrho):
    """Each compiled gain-kernel geometry gives the oracle's result (FP32 tolerance)."""
    _require_gpu()
    from paper_1903_03056_amd import CollisionPlan, tile_candidates
    print(f"[case] tiles N={N}", flush=True)
    rng = np.random.default_rng(N + 100)
    masses = (1.0, 2.0)
    f = I.draw_bimaxwellian_batch(rng, 1, 2, N, 6.0, masses, noise=1e-2).astype(np.float32).astype(np.float64)
    ref = OS.collide(f[0], _oracle_problem(masses, 0.74, 6.0, N, M, nrho))
    for tile in tile_candidates(N, "f32"):
        print(f"[case] tile {tile}", flush=True)
        plan = CollisionPlan(masses, N, 6.0, M, nrho, omega=0.74, precision="f32", tile=tile)
        assert _rel(_run(plan, f)[0], ref) <= 1e-5, tile


def _uneven_group():
    from paper_1903_03056_amd import CollisionGroup, CollisionPlan
    masses = (1.0, 2.0, 4.0)
    shapes = [(24, 3), (32, 2), (48, 1)]
    plans = [CollisionPlan(masses, N, 6.0, 6, 4, omega=0.74, precision="f32") for N, _ in shapes]
    rng = np.random.default_rng(4)
    fs = [I.draw_bimaxwellian_batch(rng, b, 3, N, 6.0, masses).astype(np.float32) for N, b in shapes]
    return masses, shapes, plans, CollisionGroup(plans), fs


def test_group_uneven_batch():
    """N = 24, 32 and 48 nodes of 3 species in one group call: one node per class
    against the oracle, every class equal bit for bit to its plan alone."""
    _require_gpu()
    print("[case] group uneven", flush=True)
    masses, shapes, plans, group, fs = _uneven_group()
    ft = [torch.tensor(f, device="cuda") for f in fs]
    outs = group.collide(ft)
    torch.cuda.synchronize()
    for (N, b), plan, f, q, x in zip(shapes, plans, fs, outs, ft):
        alone = plan.collide(x)
        torch.cuda.synchronize()
        assert torch.equal(alone, q), N
        ref = OS.collide(f[0].astype(np.float64), _oracle_problem(masses, 0.74, 6.0, N, 6, 4))
        assert _rel(q[0].double().cpu().numpy(), ref) <= 1e-5, N


def test_group_graph_replays():
    """The captured graph replayed several times, with new inputs written eagerly
    between replays; every replay equals the eager group call on the same inputs."""
    _require_gpu()
    print("[case] group graph", flush=True)
    masses, shapes, plans, group, fs = _uneven_group()
    ft = [torch.tensor(f, device="cuda") for f in fs]
    graph, gout = group.capture(ft)
    rng = np.random.default_rng(99)
    for rep in range(3):
        for x in ft:
            x.mul_(float(rng.uniform(0.5, 1.5)))
            x.add_(torch.rand_like(x) * 1e-3)
        torch.cuda.synchronize()
        graph.launch()
        graph.stream.synchronize()
        eager = group.collide(ft)
        torch.cuda.synchronize()
        for a, b in zip(gout, eager):
            assert torch.equal(a, b), rep
    graph.close()


def test_autotuner_picks_a_candidate(tmp_path, monkeypatch):
    _require_gpu()
    print("[case] autotune", flush=True)
    from paper_1903_03056_amd import CollisionPlan, tile_candidates, vhs_kernel
    from paper_1903_03056_amd import autotune
    monkeypatch.setenv("DGFS_TUNE_CACHE", str(tmp_path / "tiles.json"))
    masses = (1.0, 2.0)
    best = autotune.best_tile(masses, 32, 6.0, 12, 16, vhs_kernel(masses, 0.74), "f32", batch=8, reps=2)
    assert best in tile_candidates(32, "f32")
    assert (tmp_path / "tiles.json").exists()
    plan = CollisionPlan(masses, 32, 6.0, 12, 16, omega=0.74, precision="f32", tile="auto")
    assert plan.tile == best


# ------------------------------------------------------ plain FP64 path
@pytest.mark.parametrize("N,M,nrho", [(16, 12, 8), (24, 6, 6)])
def test_plain_fp64_path_vs_oracle_and_fused(N, M, nrho):
    """The plain per-point FP64 path (unfused, all directions per ordered pair) equals
    the oracle to 1e-12 and the fused FP64 path to 1e-13."""
    _require_gpu()
    print(f"[case] plain fp64 N={N}", flush=True)
    rng = np.random.default_rng(17)
    masses = (1.0, 2.0)
    f = I.draw_bimaxwellian_batch(rng, 2, 2, N, 6.0, masses, noise=1e-2)
    plan = _plan(masses, N, 6.0, M, nrho, 0.74, "f64")
    ft = torch.tensor(f, device="cuda")
    Qp = plan.collide_plain(ft)
    Qf = plan.collide(ft)
    torch.cuda.synchronize()
    qp, qf = Qp.cpu().numpy(), Qf.cpu().numpy()
    prob = _oracle_problem(masses, 0.74, 6.0, N, M, nrho)
    for b in range(2):
        assert _rel(qp[b], OS.collide(f[b], prob)) <= 1e-12
        assert _rel(qf[b], qp[b]) <= 1e-13


def test_plain_path_rejects_fp32_plan():
    _require_gpu()
    from paper_1903_03056_amd._lib import DgfsError
    plan = _plan((1.0, 2.0), 16, 5.0, 6, 8, 1.0, "f32")
    with pytest.raises(DgfsError):
        plan.collide_plain(torch.zeros((1, 2, 16, 16, 16), dtype=torch.float32, device="cuda"))


# --------------------------------------------------------------- conservation
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_conserve_matches_oracle_projection(precision):
    """FP64 projection on the device against the oracle's projection of the same raw
    result; the projected result conserves to 1e-12."""
    _require_gpu()
    print(f"[case] conserve {precision}", flush=True)
    rng = np.random.default_rng(13)
    masses = (1.0, 2.0)
    f = I.draw_bimaxwellian_batch(rng, 3, 2, 16, 6.0, masses, noise=1e-2)
    plan = _plan(masses, 16, 6.0, 12, 8, 0.74, precision)
    dt = torch.float64 if precision == "f64" else torch.float32
    Qr = plan.collide(torch.tensor(f, dtype=dt, device="cuda"))
    Qc = plan.conserve(Qr)
    torch.cuda.synchronize()
    raw = Qr.double().cpu().numpy()
    got = Qc.cpu().numpy()
    for b in range(3):
        ref = OM.conserve(raw[b], masses, (6.0, 6.0))
        assert np.abs(got[b] - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.all(OM.conservation_residual(got[b], masses, (6.0, 6.0)) <= 1e-12)


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_conserve_update_is_euler_step_of_projection(precision):
    """dgfs_conserve_update: f <- f + dt * projection(Q) in FP64 arithmetic, stored in the
    plan's precision, against the oracle's projection of the same raw result (within one
    unit in the last place of the stored type, plus dt times the projection's own 1e-12
    relative tolerance)."""
    _require_gpu()
    print(f"[case] conserve_update {precision}", flush=True)
    rng = np.random.default_rng(17)
    masses = (1.0, 2.0, 4.0)
    f = I.draw_bimaxwellian_batch(rng, 3, 3, 16, 6.0, masses, noise=1e-2)
    plan = _plan(masses, 16, 6.0, 12, 8, 0.74, precision)
    dt_t = torch.float64 if precision == "f64" else torch.float32
    np_t = np.float64 if precision == "f64" else np.float32
    ft = torch.tensor(f, dtype=dt_t, device="cuda")
    Qr = plan.collide(ft)
    f0 = ft.double().cpu().numpy()
    raw = Qr.double().cpu().numpy()
    dt = 0.01
    plan.relax_step(ft, Qr, dt)
    torch.cuda.synchronize()
    got = ft.cpu().numpy()
    for b in range(3):
        proj = OM.conserve(raw[b], masses, (6.0,) * 3)
        ref = (f0[b] + dt * proj).astype(np_t)
        tol = np.spacing(np.abs(ref)).astype(np.float64) + dt * 1e-12 * np.abs(proj).max()
        assert np.all(np.abs(got[b].astype(np.float64) - ref.astype(np.float64)) <= tol)


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_large_mass_ratio(precision, tol):
    """Masses (1, 4, 20) (mass ratio 20: a, b = 1/21, 20/21 for the light-heavy pair),
    N = 24, M = 12, N_rho = 12, L = 6, omega = 0.74."""
    _require_gpu()
    print(f"[case] mass ratio 20 {precision}", flush=True)
    rng = np.random.default_rng(23)
    masses = (1.0, 4.0, 20.0)
    f = I.draw_bimaxwellian_batch(rng, 2, 3, 24, 6.0, masses)
    Q = _run(_plan(masses, 24, 6.0, 12, 12, 0.74, precision), f)
    prob = _oracle_problem(masses, 0.74, 6.0, 24, 12, 12)
    for b in range(2):
        ref = OS.collide(f[b].astype(np.float32).astype(np.float64) if precision == "f32" else f[b], prob)
        assert _rel(Q[b], ref) <= tol
