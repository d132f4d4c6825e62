"""The matrix-core gain (geometry (2, 0): FP32, VHS kernels, N = 32) on the inputs that
stress its arithmetic: every FP16 operand is a split of a value scaled per (node,
species) by a power of two, so results must not depend on the magnitude of f, on the
two species' magnitudes differing by orders, or on the batch's layout over the XCDs.

Tolerances as in the other FP32 parity tests: 1e-5 relative L-inf against the FP64
oracle (rel = max over (node, species) of max_n |Q - Q_ref| / max_n |Q_ref|)."""
import numpy as np
import pytest

from oracle import spectral as OS
from synth import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MASSES = (1.0, 2.0)
N, L, M, NRHO, OMEGA = 32, 6.0, 6, 4, 0.74


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rel(q, ref):
    q = q.reshape(-1, N ** 3)
    ref = ref.reshape(q.shape)
    return float(np.max(np.abs(q - ref).max(axis=1) / np.abs(ref).max(axis=1)))


def _plan(tile=(2, 0)):
    from paper_1903_03056_amd import CollisionPlan
    return CollisionPlan(MASSES, N, L, M, NRHO, omega=OMEGA, precision="f32", tile=tile)


def _collide(plan, f):
    Q = plan.collide(torch.tensor(f, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    return Q.double().cpu().numpy()


def test_matrix_core_is_the_default_and_matches_oracle():
    """The default N = 32 FP32 geometry is (2, 0); two noisy bi-Maxwellian nodes agree with
    the oracle."""
    _require_gpu()
    from paper_1903_03056_amd import tile_candidates
    print("[case] matrix-core default N=32", flush=True)
    assert tile_candidates(N, "f32")[0] == (2, 0)
    f = I.draw_bimaxwellian_batch(np.random.default_rng(21), 2, 2, N, L, MASSES, noise=1e-2).astype(np.float32)
    from paper_1903_03056_amd import CollisionPlan
    plan = CollisionPlan(MASSES, N, L, M, NRHO, omega=OMEGA, precision="f32")
    Q = _collide(plan, f)
    prob = OS.vhs_problem(MASSES, OMEGA, L, N, M, NRHO)
    for b in range(2):
        ref = OS.collide(f[b].astype(np.float64), prob)
        err = _rel(Q[b], ref)
        print(f"node {b}: {err:.3e}", flush=True)
        assert err <= 1e-5


@pytest.mark.parametrize("scale", [1e-15, 1e-6, 1e9, 1e17])
def test_matrix_core_scale_invariance(scale):
    """Q is quadratic in f: Q(s f) = s^2 Q(f).  The per-(node, species) power-of-two scaling
    of the split operands makes the matrix-core result at s f equal s^2 times the result at
    f up to rounding, from 1e-15 (below FP16's range without the scaling) to 1e17 (far
    above it); s^2 Q stays in FP32's normal range."""
    _require_gpu()
    print(f"[case] matrix-core scale {scale:g}", flush=True)
    f = I.draw_bimaxwellian_batch(np.random.default_rng(22), 2, 2, N, L, MASSES, noise=1e-2).astype(np.float32)
    plan = _plan()
    Q1 = _collide(plan, f)
    Qs = _collide(plan, (f.astype(np.float64) * scale).astype(np.float32)) / (scale * scale)
    err = _rel(Qs, Q1)
    print(f"relative difference {err:.3e}", flush=True)
    assert np.all(np.isfinite(Qs))
    assert err <= 1e-5


def test_matrix_core_species_of_different_magnitudes():
    """Species 1 at 1e-4 of species 0's magnitude (each species is scaled on its own): the
    summed result of both species against the oracle."""
    _require_gpu()
    print("[case] matrix-core species magnitudes", flush=True)
    f = I.draw_bimaxwellian_batch(np.random.default_rng(23), 1, 2, N, L, MASSES, noise=1e-2)
    f[:, 1] *= 1e-4
    f = f.astype(np.float32)
    Q = _collide(_plan(), f)
    ref = OS.collide(f[0].astype(np.float64), OS.vhs_problem(MASSES, OMEGA, L, N, M, NRHO))
    err = _rel(Q[0], ref)
    print(f"relative L-inf {err:.3e}", flush=True)
    assert err <= 1e-5


def test_matrix_core_zero_input_and_ragged_batches():
    """f = 0 gives Q = 0 exactly; in a batch of 37 nodes (not a multiple of the 32 nodes one
    pass of the XCD-interleaved work items covers) every node equals its result alone, bit
    for bit."""
    _require_gpu()
    print("[case] matrix-core zero and ragged", flush=True)
    plan = _plan()
    z = _collide(plan, np.zeros((3, 2, N, N, N), dtype=np.float32))
    assert np.array_equal(z, np.zeros_like(z))
    f = I.draw_bimaxwellian_batch(np.random.default_rng(24), 37, 2, N, L, MASSES, noise=1e-2).astype(np.float32)
    Q = _collide(plan, f)
    for b in (0, 8, 31, 32, 36):
        alone = _collide(plan, f[b:b + 1])
        assert np.array_equal(alone[0], Q[b]), b


def test_matrix_core_rejected_where_it_does_not_apply():
    """The geometry needs FP32, N = 32, alpha = 1 and the circular form; elsewhere the
    library reports DGFS_EUNSUPPORTED, and VSS or dealiased plans at N = 32 default to an
    FFT geometry."""
    from paper_1903_03056_amd import CollisionPlan, check_problem, vhs_kernel, vss_kernel
    from paper_1903_03056_amd._lib import DGFS_EUNSUPPORTED, DGFS_OK
    k = vhs_kernel(MASSES, OMEGA)
    assert check_problem(MASSES, L, 32, 12, 16, k, tile=(2, 0)) == DGFS_OK
    assert check_problem(MASSES, L, 32, 12, 16, vss_kernel(MASSES, 0.8, 1.4), tile=(2, 0)) == DGFS_EUNSUPPORTED
    assert check_problem(MASSES, L, 32, 12, 16, k, precision="f64", tile=(2, 0)) == DGFS_EUNSUPPORTED
    assert check_problem(MASSES, L, 24, 12, 12, k, tile=(2, 0)) == DGFS_EUNSUPPORTED
    assert check_problem(MASSES, L, 32, 12, 16, k, tile=(2, 0), dealias=True) == DGFS_EUNSUPPORTED
    _require_gpu()
    print("[case] matrix-core rejection", flush=True)
    # a VSS plan at N = 32 with the default geometry runs (FFT geometry) and matches the
    # oracle to the FP32 tolerance
    kv = vss_kernel(MASSES, 0.8, 1.4)
    plan = CollisionPlan(MASSES, 32, L, 6, 4, kernel=kv, precision="f32")
    f = I.draw_bimaxwellian_batch(np.random.default_rng(25), 1, 2, N, L, MASSES, noise=1e-2).astype(np.float32)
    Q = _collide(plan, f)
    prob = OS.Problem(masses=MASSES, L=L, N=32, M=6, nrho=4, kernel=kv)
    ref = OS.collide_pairs(f[0].astype(np.float64), prob).sum(axis=1)
    err = _rel(Q[0], ref)
    print(f"VSS default geometry: {err:.3e}", flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("noise", [0.5, 1.0])
def test_matrix_core_rough_inputs(noise):
    """Grid noise of half and all of the peak (clipped at zero): the alternating sums behind
    the correction terms are then far from zero.  Both the matrix-core and the FFT
    geometry against the oracle, each within the FP32 bound."""
    _require_gpu()
    print(f"[case] matrix-core rough input, noise {noise}", flush=True)
    f = I.draw_bimaxwellian_batch(np.random.default_rng(31), 1, 2, N, L, MASSES, noise=noise).astype(np.float32)
    ref = OS.collide(f[0].astype(np.float64), OS.vhs_problem(MASSES, OMEGA, L, N, M, NRHO))
    errs = {}
    for tile in ((2, 0), (2, 1)):
        errs[tile] = _rel(_collide(_plan(tile), f)[0], ref)
    print(f"matrix cores {errs[(2, 0)]:.3e}, FFT {errs[(2, 1)]:.3e}", flush=True)
    assert errs[(2, 0)] <= 1e-5 and errs[(2, 1)] <= 1e-5


def test_matrix_core_repeats_bit_for_bit():
    """The same batch three times in a row gives the same bits: an operand read by a matrix
    product before the instruction that forms it has landed would show up here as
    rounding-level differences between runs."""
    _require_gpu()
    print("[case] matrix-core run-to-run", flush=True)
    plan = _plan()
    f = I.draw_bimaxwellian_batch(np.random.default_rng(26), 37, 2, N, L, MASSES, noise=1e-2).astype(np.float32)
    runs = [_collide(plan, f) for _ in range(3)]
    assert np.array_equal(runs[0], runs[1]) and np.array_equal(runs[0], runs[2])


def test_matrix_core_non_antipodal_design():
    """The 24-point design (not antipodal: one class per ordered pair, 24 directions each)
    with two radial points, against the oracle."""
    _require_gpu()
    print("[case] matrix-core M=24", flush=True)
    from paper_1903_03056_amd import CollisionPlan
    f = I.draw_bimaxwellian_batch(np.random.default_rng(27), 2, 2, N, L, MASSES, noise=1e-2).astype(np.float32)
    plan = CollisionPlan(MASSES, N, L, 24, 2, omega=OMEGA, precision="f32", tile=(2, 0))
    Q = _collide(plan, f)
    prob = OS.vhs_problem(MASSES, OMEGA, L, N, 24, 2)
    for b in range(2):
        err = _rel(Q[b], OS.collide(f[b].astype(np.float64), prob))
        print(f"node {b}: {err:.3e}", flush=True)
        assert err <= 1e-5
