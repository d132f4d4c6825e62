"""Serving scheduler on the CPU: trace generation, HBM-budget admission, slot compaction
and continuous batching, with a fake device backend whose 'step' is a known map."""
import math

import numpy as np
import pytest

from paper_1903_03056_amd import serve as S


class FakePool:
    """Slots in host memory; a step applies f <- f + dt * (1 - f) to slots [0, n).
    ready() turns true `latency` polls after a launch."""

    BYTES_PER_SLOT = 1000
    WS_BYTES = 500

    def __init__(self, key, latency):
        self.dt = key[2]
        self.cap = 0
        self.f = None
        self.latency = latency
        self.wait = 0
        self.launch_sizes = []

    def bytes_for(self, cap):
        return 0 if cap == 0 else cap * self.BYTES_PER_SLOT + self.WS_BYTES

    def resize(self, cap, live):
        if cap == 0:
            self.f, self.cap = None, 0
            return
        f = np.zeros((cap, 3))
        if live:
            f[:live] = self.f[:live]
        self.f, self.cap = f, cap

    def insert(self, slot, staged):
        self.f[slot] = staged

    def move(self, dst, src):
        self.f[dst] = self.f[src]

    def read(self, slot):
        return self.f[slot].copy()

    def launch(self, n):
        assert 0 < n <= self.cap
        self.f[:n] = self.f[:n] + self.dt * (1.0 - self.f[:n])
        self.launch_sizes.append(n)
        self.wait = self.latency

    def ready(self):
        if self.wait > 0:
            self.wait -= 1
            return False
        return True

    def sync(self):
        self.wait = 0


class FakeBackend:
    def __init__(self, latency=0):
        self.latency = latency
        self.pools = {}

    def new_pool(self, key):
        self.pools[key] = FakePool(key, self.latency)
        return self.pools[key]

    def stage(self, payload):
        # a small per-request payload that identifies the request
        return np.array([float(payload.shape[0]), float(payload.shape[1]), float(payload.sum())])


def _expected(req, staged):
    x = staged.copy()
    for _ in range(req.steps):
        x = x + req.dt * (1.0 - x)
    return x


def _trace(n=60, rate=1e6, seed=3, steps=7):
    return S.make_trace(n, rate, seed, steps=steps, Ns=(4, 6))


def test_trace_is_seeded_and_has_the_stated_mix():
    a = S.make_trace(2000, 2000.0, 5)
    b = S.make_trace(2000, 2000.0, 5)
    c = S.make_trace(2000, 2000.0, 6)
    assert [(r.t_arrive, r.masses, r.N) for r in a] == [(r.t_arrive, r.masses, r.N) for r in b]
    assert [(r.t_arrive, r.masses, r.N) for r in a] != [(r.t_arrive, r.masses, r.N) for r in c]
    gaps = np.diff([0.0] + [r.t_arrive for r in a])
    assert np.all(gaps > 0)
    assert abs(gaps.mean() * 2000.0 - 1.0) < 0.1          # mean gap 1/rate (4.5 sigma)
    assert {len(r.masses) for r in a} == {2, 3}
    for r in a:
        assert len(set(r.masses)) == len(r.masses) and set(r.masses) <= set(S.MASS_POOL)
        assert list(r.masses) == sorted(r.masses)
        assert r.N in S.N_CHOICES and r.steps == 50 and r.dt == 0.01
    counts = np.bincount([S.N_CHOICES.index(r.N) for r in a], minlength=4)
    assert counts.min() > 400                              # uniform over the 4 grids


def test_initial_state_is_seeded_per_request():
    r = S.make_trace(3, 10.0, 5, Ns=(8,))
    x0, x1 = S.initial_state(r[0]), S.initial_state(r[0])
    assert x0.dtype == np.float32 and x0.shape == (len(r[0].masses), 8, 8, 8)
    np.testing.assert_array_equal(x0, x1)
    assert not np.array_equal(S.initial_state(r[1])[0], x0[0])


@pytest.mark.parametrize("latency", [0, 3])
def test_every_request_keeps_its_own_state_through_compaction(latency):
    """Requests join and leave pools at different steps; each final state is its own
    initial data advanced exactly `steps` times."""
    trace = _trace()
    for k, r in enumerate(trace):
        r.steps = 3 + k % 5                # requests leave at different steps
    srv = S.Server(backend=FakeBackend(latency), budget_bytes=10 ** 9, keep_final=True)
    staged, _ = srv.warm(trace)
    res = srv.run(trace, staged, realtime=False)
    assert res["requests"] == len(trace)
    for r in trace:
        np.testing.assert_array_equal(r.final, _expected(r, staged[r.rid]))
        assert r.t_done >= r.t_admit
    assert srv.budget.used == 0                            # every pool returned its bytes


def test_budget_defers_and_never_exceeds():
    """A budget that fits one small pool: requests wait for memory, none is dropped, and
    the bytes held never exceed the limit."""
    trace = _trace(40)
    one_pool = FakePool.BYTES_PER_SLOT * 4 + FakePool.WS_BYTES
    srv = S.Server(backend=FakeBackend(1), budget_bytes=one_pool, keep_final=True)
    staged, _ = srv.warm(trace)
    res = srv.run(trace, staged, realtime=False)
    assert res["deferrals"] > 0
    assert srv.budget.peak <= one_pool
    for r in trace:
        np.testing.assert_array_equal(r.final, _expected(r, staged[r.rid]))
    for pool in srv.backend.pools.values():
        assert max(pool.launch_sizes) <= 4
    assert srv.budget.used == 0


def test_request_that_cannot_fit_alone_raises():
    trace = _trace(3)
    srv = S.Server(backend=FakeBackend(), budget_bytes=FakePool.BYTES_PER_SLOT)
    staged, _ = srv.warm(trace)
    with pytest.raises(RuntimeError, match="does not fit"):
        srv.run(trace, staged, realtime=False)


def test_late_arrivals_join_running_pools():
    """Continuous batching: with arrivals spread in time, requests enter a pool while
    earlier ones are still stepping, so launches carry requests at different progress."""
    trace = S.make_trace(40, 4000.0, 11, steps=30, Ns=(4,))
    srv = S.Server(backend=FakeBackend(latency=2), budget_bytes=10 ** 9, keep_final=True)
    staged, _ = srv.warm(trace)
    res = srv.run(trace, staged, realtime=True)
    sizes = [n for p in srv.backend.pools.values() for n in p.launch_sizes]
    total_steps = sum(r.steps for r in trace)
    assert sum(sizes) == total_steps                      # every launch advanced exactly its slots
    assert res["launches"] < total_steps                  # requests shared launches
    # some request entered a pool after another of the same pool had started
    by_pool = {}
    for r in trace:
        by_pool.setdefault(r.key, []).append(r)
    assert any(a.t_admit < b.t_admit < a.t_done for rs in by_pool.values() for a in rs for b in rs)
    for r in trace:
        np.testing.assert_array_equal(r.final, _expected(r, staged[r.rid]))
    assert math.isfinite(res["latency_p99_s"]) and res["latency_p99_s"] >= res["latency_p50_s"]


def test_grown_capacity_doubles_from_four():
    assert S.grown_capacity(0, 1) == 4
    assert S.grown_capacity(4, 5) == 8
    assert S.grown_capacity(8, 33) == 64
    assert S.grown_capacity(16, 3) == 16
