"""GPU parity of the 1-D DG slab (Sec. 5): the transport kernel against the oracle's
nodal DG operator at the full 64 x 4 slab size, SSP-RK2 steps of transport plus
projected collisions on a small slab against the oracle's, and mass conservation
between two diffuse walls at full size."""
import numpy as np
import pytest

from oracle import dg, spectral as OS, stepping as OT
from synth import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BCS = {
    "inflow": dict(kind="inflow", n=(1.0, 0.6), u=(0.3, 0.0, 0.0), T=1.0),
    "inflow_r": dict(kind="inflow", n=(0.8, 0.5), u=(-0.2, 0.0, 0.0), T=1.3),
    "wall_l": dict(kind="wall", u=(0.0, -0.3, 0.0), T=0.9),
    "wall_r": dict(kind="wall", u=(0.0, 0.3, 0.0), T=1.2),
}


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _obc(spec):
    return dg.Boundary(spec["kind"], u=tuple(spec["u"]), T=spec["T"], n=tuple(spec.get("n", ())))


def _state(rng, nodes, masses, N, L):
    f = I.draw_bimaxwellian_batch(rng, nodes, len(masses), N, (L,) * len(masses), masses, noise=1e-2)
    return f


def _plan(masses, N, L, M, nrho, precision):
    from paper_1903_03056_amd import CollisionPlan
    return CollisionPlan(masses, N, L, M, nrho, omega=0.74, precision=precision)


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 2e-6)])
@pytest.mark.parametrize("sides", [("inflow", "wall_r"), ("wall_l", "inflow_r")])
def test_transport_full_size(precision, tol, sides):
    """64 elements x 4 GLL nodes, N = 32, two species, collisions off: one Euler step
    f + dt T(f) against the oracle, relative to max |f|; the change against the oracle's
    change, relative to its maximum."""
    _require_gpu()
    from paper_1903_03056_amd import Slab
    print(f"[case] slab transport {precision} {sides}", flush=True)
    masses, N, L, Ne, K = (1.0, 2.0), 32, 6.0, 64, 4
    plan = _plan(masses, N, L, 12, 16, precision)
    slab = Slab(plan, 0.0, 1.0, Ne, K, BCS[sides[0]], BCS[sides[1]], collide=False)
    f = _state(np.random.default_rng(21), Ne * K, masses, N, L)
    dt = torch.float64 if precision == "f64" else torch.float32
    ft = torch.tensor(f, dtype=dt, device="cuda")
    f0 = ft.double().cpu().numpy()
    slab.step(ft, 1e-3, 1, scheme="euler")
    got = ft.double().cpu().numpy().reshape(Ne, K, 2, N, N, N)
    o = dg.Slab(0.0, 1.0, Ne, K, masses, N, (L, L), _obc(BCS[sides[0]]), _obc(BCS[sides[1]]))
    F = f0.reshape(Ne, K, 2, N, N, N)
    ref = F + 1e-3 * o.transport(F)
    rel = float(np.abs(got - ref).max() / np.abs(ref).max())
    drel = float(np.abs((got - F) - (ref - F)).max() / np.abs(ref - F).max())
    print(f"state {rel:.3e}, change {drel:.3e}", flush=True)
    assert rel <= tol
    assert drel <= (1e-10 if precision == "f64" else 1e-4)


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
@pytest.mark.parametrize("sides", [("inflow", "inflow_r"), ("wall_l", "wall_r")])
def test_ssprk2_with_collisions_small_slab(precision, tol, sides):
    """3 elements x 3 GLL nodes, N = 16, M = 6, N_rho = 8: one SSP-RK2 step of transport
    plus the projected collision operator against the oracle's, as states (relative to
    max |f|) and as changes f - f0 (relative to the largest change)."""
    _require_gpu()
    from paper_1903_03056_amd import Slab
    print(f"[case] slab ssprk2 {precision} {sides}", flush=True)
    masses, N, L, M, nrho, Ne, K = (1.0, 2.0), 16, 5.0, 6, 8, 3, 3
    plan = _plan(masses, N, L, M, nrho, precision)
    slab = Slab(plan, 0.0, 0.5, Ne, K, BCS[sides[0]], BCS[sides[1]])
    f = _state(np.random.default_rng(22), Ne * K, masses, N, L)
    dtp = torch.float64 if precision == "f64" else torch.float32
    ft = torch.tensor(f, dtype=dtp, device="cuda")
    F = ft.double().cpu().numpy().reshape(Ne, K, 2, N, N, N)
    slab.step(ft, 2e-3, 1)
    got = ft.double().cpu().numpy().reshape(F.shape)
    o = dg.Slab(0.0, 0.5, Ne, K, masses, N, (L, L), _obc(BCS[sides[0]]), _obc(BCS[sides[1]]))
    prob = OS.vhs_problem(masses, 0.74, L, N, M, nrho)
    ref = OT.ssprk2(F, dg.slab_rhs(o, prob), 2e-3, 1)
    rel = float(np.abs(got - ref).max() / np.abs(ref).max())
    drel = float(np.abs((got - F) - (ref - F)).max() / np.abs(ref - F).max())
    print(f"state relative L-inf {rel:.3e}; change relative L-inf {drel:.3e}", flush=True)
    assert rel <= tol
    assert drel <= (1e-10 if precision == "f64" else 1e-4)


def test_walls_conserve_mass_full_size():
    """64 x 4 nodes between two diffuse walls, N = 32, M = 12, N_rho = 16, FP64, collisions
    on: two Euler steps keep each species' GLL-weighted mass to 1e-12 (the walls pass no
    net mass and the projection conserves it at every node); SSP-RK2 likewise."""
    _require_gpu()
    from paper_1903_03056_amd import Slab
    print("[case] slab walls mass", flush=True)
    masses, N, L, Ne, K = (1.0, 2.0), 32, 6.0, 64, 4
    plan = _plan(masses, N, L, 12, 16, "f64")
    slab = Slab(plan, 0.0, 1.0, Ne, K, BCS["wall_l"], BCS["wall_r"])
    o = dg.Slab(0.0, 1.0, Ne, K, masses, N, (L, L), _obc(BCS["wall_l"]), _obc(BCS["wall_r"]))
    f = _state(np.random.default_rng(23), Ne * K, masses, N, L)
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    m0 = o.mass(f.reshape(Ne, K, 2, N, N, N))
    slab.step(ft, 1e-3, 2, scheme="euler")
    m1 = o.mass(ft.cpu().numpy().reshape(Ne, K, 2, N, N, N))
    slab.step(ft, 1e-3, 2, scheme="ssprk2")
    m2 = o.mass(ft.cpu().numpy().reshape(Ne, K, 2, N, N, N))
    print(f"mass {m0} -> {m1} -> {m2}", flush=True)
    np.testing.assert_allclose(m1, m0, rtol=1e-12)
    np.testing.assert_allclose(m2, m0, rtol=1e-12)


def test_slab_errors():
    _require_gpu()
    from paper_1903_03056_amd import Slab
    from paper_1903_03056_amd._lib import DgfsError
    plan = _plan((1.0, 2.0), 16, 5.0, 6, 4, "f64")
    with pytest.raises(DgfsError):
        Slab(plan, 0.0, 1.0, 4, 9, BCS["inflow"], BCS["wall_r"])          # K > 8
    with pytest.raises(DgfsError):
        Slab(plan, 1.0, 0.0, 4, 3, BCS["inflow"], BCS["wall_r"])          # x1 < x0
    with pytest.raises(DgfsError):
        Slab(plan, 0.0, 1.0, 4, 3, BCS["inflow"], dict(kind="wall", u=(0.1, 0, 0), T=1.0))   # wall moving in x
    slab = Slab(plan, 0.0, 1.0, 2, 2, BCS["inflow"], BCS["wall_r"])
    with pytest.raises(DgfsError):
        slab.step(torch.zeros((4, 2, 16, 16, 16), dtype=torch.float64, device="cuda"), 1e-3, 1,
                  workspace=torch.empty(256, dtype=torch.uint8, device="cuda"))


def test_many_steps_stay_bounded_fp32():
    """The bench configuration (64 x 4 nodes between diffuse walls, N = 32, M = 12,
    N_rho = 16, FP32) over 20 SSP-RK2 steps at dt = 2e-4 (transport CFL 0.077) from
    noise-free bi-Maxwellians: finite, the maximum within 1.2 x its start, each species'
    mass kept to 1e-5.  (A uniform noise floor over the whole velocity box would be a hot
    tail that the diffuse walls re-emit as slow particles, piling up at the wall nodes:
    the model's answer for that input, not an instability.)

    Positivity: the nodal data are independent draws per node, so each element's cubic
    interpolant oscillates and the unlimited DG transport (Sec. 5) undershoots: the
    oracle's transport alone on these inputs reaches min f = -0.205 max f_0 after 20
    steps (tests/golden/oracle_slab_transport_min.json).  The device's minimum after each
    step stays within 0.01 max f_0 of that sequence (the collision term moves f by about
    dt |Q| per stage), and above -0.25 max f_0."""
    _require_gpu()
    from paper_1903_03056_amd import Slab
    print("[case] slab 20 steps fp32", flush=True)
    masses, N, L, Ne, K = (1.0, 2.0), 32, 6.0, 64, 4
    plan = _plan(masses, N, L, 12, 16, "f32")
    slab = Slab(plan, 0.0, 1.0, Ne, K, dict(kind="wall", u=(0.0, -0.3, 0.0), T=1.0),
                dict(kind="wall", u=(0.0, 0.3, 0.0), T=1.0))
    o = dg.Slab(0.0, 1.0, Ne, K, masses, N, (L, L), dg.Boundary("wall", u=(0.0, -0.3, 0.0), T=1.0),
                dg.Boundary("wall", u=(0.0, 0.3, 0.0), T=1.0))
    f = I.draw_bimaxwellian_batch(np.random.default_rng(2), Ne * K, 2, N, (L, L), masses).astype(np.float32)
    ft = torch.tensor(f, device="cuda")
    m0 = o.mass(f.astype(np.float64).reshape(Ne, K, 2, N, N, N))
    ws = torch.empty(slab.workspace_bytes(), dtype=torch.uint8, device="cuda")
    lows = []
    for _ in range(20):
        slab.step(ft, 2e-4, 1, workspace=ws)
        lows.append(float(ft.min()) / float(f.max()))
    g = ft.double().cpu().numpy()
    m1 = o.mass(g.reshape(Ne, K, 2, N, N, N))
    print(f"mass {m0} -> {m1}; min {g.min():.3e} max {g.max():.3e} (start {f.max():.3e})", flush=True)
    print(f"min f / max f0 after each step: {np.array2string(np.array(lows), precision=3)}", flush=True)
    assert np.isfinite(g).all()
    assert g.max() < 1.2 * f.max()
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "oracle_slab_transport_min.json")) as fh:
        ref = np.array(json.load(fh)["min_over_max0"])
    print(f"oracle transport alone:           {np.array2string(ref, precision=3)}", flush=True)
    assert np.all(np.abs(np.array(lows) - ref) <= 0.01)
    assert min(lows) >= -0.25
    np.testing.assert_allclose(m1, m0, rtol=1e-5)
