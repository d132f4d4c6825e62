"""Serving on the device: each request's result is the same alone and in the mix, and a
served request follows the oracle's forward-Euler trajectory."""
import numpy as np
import pytest

from oracle import moments as OM, spectral as OS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_alone_equals_in_mix_and_follows_oracle():
    """12 requests over N in {16, 24} and 2-3 species, 4 Euler steps each, served together
    with staggered step counts (so slots are compacted while others run), then each alone
    in a fresh server: the final states agree bit for bit (every node's arithmetic is
    independent of its batch and slot).  Two of them are checked against the oracle's
    trajectory f <- f + dt * projection(Q_fast) in FP64: relative L-inf <= 1e-5."""
    _require_gpu()
    from paper_1903_03056_amd import serve as S
    print("[case] serve alone vs mix", flush=True)
    trace = S.make_trace(12, 1e6, 21, steps=4, Ns=(16, 24))
    for k, r in enumerate(trace):
        r.steps = 2 + k % 3
    backend = S.DeviceBackend()
    mix = S.Server(backend=backend, budget_bytes=16 << 30, keep_final=True)
    staged, _ = mix.warm(trace)
    mix.run(trace, staged, realtime=False)
    finals = {r.rid: r.final for r in trace}
    for r in trace:
        alone = S.Server(backend=backend, budget_bytes=16 << 30, keep_final=True)
        r.final = None
        alone.run([r], {r.rid: staged[r.rid]}, realtime=False)
        np.testing.assert_array_equal(r.final, finals[r.rid], err_msg=f"request {r.rid}")

    checked = 0
    for r in trace:
        if r.N != 16 or checked == 2:
            continue
        print(f"[case] serve oracle trajectory request {r.rid} masses={r.masses}", flush=True)
        prob = OS.vhs_problem(r.masses, S.OMEGA, S.L_BOX, r.N, S.M_DESIGN, r.N // 2)
        Ls = (S.L_BOX,) * len(r.masses)
        f = S.initial_state(r).astype(np.float64)
        for _ in range(r.steps):
            f = f + r.dt * OM.conserve(OS.collide(f, prob), r.masses, Ls)
        got = finals[r.rid].astype(np.float64)
        for i in range(len(r.masses)):
            assert np.abs(got[i] - f[i]).max() <= 1e-5 * np.abs(f[i]).max()
        checked += 1
    assert checked == 2


def test_ssprk2_serving_follows_oracle():
    """Serving with SSP-RK2 steps (dgfs_relax per pool step): four N = 16 requests of 3
    steps served together; two follow the oracle's SSP-RK2 trajectory of the projected
    operator within 1e-5 relative L-inf, and each equals its result alone bit for bit."""
    _require_gpu()
    from paper_1903_03056_amd import serve as S
    from oracle import stepping as OT
    print("[case] serve ssprk2", flush=True)
    trace = S.make_trace(4, 1e6, 31, steps=3, Ns=(16,))
    backend = S.DeviceBackend(scheme="ssprk2")
    mix = S.Server(backend=backend, budget_bytes=8 << 30, keep_final=True)
    staged, _ = mix.warm(trace)
    mix.run(trace, staged, realtime=False)
    finals = {r.rid: r.final for r in trace}
    for r in trace:
        alone = S.Server(backend=backend, budget_bytes=8 << 30, keep_final=True)
        r.final = None
        alone.run([r], {r.rid: staged[r.rid]}, realtime=False)
        np.testing.assert_array_equal(r.final, finals[r.rid], err_msg=f"request {r.rid}")
    for r in trace[:2]:
        prob = OS.vhs_problem(r.masses, S.OMEGA, S.L_BOX, r.N, S.M_DESIGN, r.N // 2)
        rhs = OT.collision_rhs(prob)
        f = OT.ssprk2(S.initial_state(r).astype(np.float32).astype(np.float64), rhs, r.dt, r.steps)
        got = finals[r.rid].astype(np.float64)
        for i in range(len(r.masses)):
            assert np.abs(got[i] - f[i]).max() <= 1e-5 * np.abs(f[i]).max()
