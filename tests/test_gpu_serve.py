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


def test_large_pool_and_N48_alone_equals_mix_and_follows_oracle():
    """A pool of 70 N = 32 requests (m = (1, 2), 3 Euler steps: more than the 64 nodes one
    workspace pass of a pool covers, so every step collides in two slices) served with
    N = 48 requests (m = (1, 2, 4) and (1, 20), 2 steps) and N = 16 and 24 ones.  Requests
    on both sides of the slice boundary and every N = 48, 16 and 24 request end bit for bit
    as they do alone; request 69 (N = 32, in the second slice) and request 101 (N = 48)
    follow the oracle's Euler trajectory of the projected operator within 1e-5 relative
    L-inf (oracle values stored at sampled grid points: tests/golden/oracle_serve_traj.npz)."""
    _require_gpu()
    import _golden as G
    from paper_1903_03056_amd import serve as S
    print("[case] serve: 70-slot N=32 pool with N=48 requests", flush=True)
    d, meta = G.load("serve_traj")
    assert (meta["L"], meta["M"], meta["omega"]) == (S.L_BOX, S.M_DESIGN, S.OMEGA)
    seed, dt = meta["seed"], meta["dt"]
    trace = [S.Request(rid=k, t_arrive=1e-4 * k, masses=(1.0, 2.0), N=32, steps=3, dt=dt, seed=seed)
             for k in range(70)]
    trace += [S.Request(rid=100, t_arrive=0.0071, masses=(1.0, 2.0, 4.0), N=48, steps=2, dt=dt, seed=seed),
              S.Request(rid=101, t_arrive=0.0072, masses=(1.0, 20.0), N=48, steps=2, dt=dt, seed=seed),
              S.Request(rid=102, t_arrive=0.0073, masses=(2.0, 4.0), N=16, steps=4, dt=dt, seed=seed),
              S.Request(rid=103, t_arrive=0.0074, masses=(1.0, 4.0, 20.0), N=24, steps=3, dt=dt, seed=seed)]
    backend = S.DeviceBackend()
    mix = S.Server(backend=backend, budget_bytes=16 << 30, keep_final=True)
    staged, _ = mix.warm(trace)
    mix.run(trace, staged, realtime=False)
    finals = {r.rid: r.final for r in trace}
    big = mix.pools[(32, (1.0, 2.0), dt)]
    assert big.dev.peak_cap >= 70 and big.launches == 3
    byid = {r.rid: r for r in trace}
    for rid in (0, 63, 64, 69, 100, 101, 102, 103):
        r = byid[rid]
        alone = S.Server(backend=backend, budget_bytes=16 << 30, keep_final=True)
        r.final = None
        alone.run([r], {rid: staged[rid]}, realtime=False)
        np.testing.assert_array_equal(r.final, finals[rid], err_msg=f"request {rid}")
    for k, req in enumerate(meta["requests"]):
        r = byid[req["rid"]]
        assert (r.N, list(r.masses), r.steps) == (req["N"], req["masses"], req["steps"])
        G.check_inputs(S.initial_state(r), d[f"r{k}_fsum"])
        got = finals[r.rid].reshape(len(r.masses), -1).astype(np.float64)
        idx, ref, fmax = d[f"r{k}_idx"], d[f"r{k}_qp"][:, 0], d[f"r{k}_qmax"]
        rel = np.array([np.abs(got[i, idx[i]] - ref[i]).max() / fmax[i] for i in range(len(r.masses))])
        print(f"request {r.rid} (N = {r.N}, {r.steps} steps): state error vs oracle {rel}", flush=True)
        assert np.all(rel <= 1e-5)
