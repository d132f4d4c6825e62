"""Continuous-batching server for spatially homogeneous relaxation problems.

Each request is an independent problem df^i/dt = sum_j Q^{ij}(f^i, f^j) (the collision
operator on one velocity grid, Sec. 4) advanced by forward-Euler steps
f <- f + dt * P(Q), P the FP64 conservation projection.  Requests differ in the velocity
resolution N and in the species set.

Scheduling:

* Requests sharing (N, masses, dt) share one *pool*: device-resident slots holding their
  distribution functions, one collision plan and one stream.  A pool advances all its
  active slots by one Euler step per launch (one batched collide + one fused
  projection/update call).
* Pools progress independently: whenever a pool's previous step has finished (its event
  has fired), the host retires the requests that reached their step count (compacting
  the pool), moves newly admitted requests into free slots and launches the next step.
  Requests join and leave at every step (continuous batching), and the pools' streams
  overlap on the device.
* Admission is in arrival order and bounded by an HBM budget: a request is admitted only
  if the bytes its pool would hold afterwards (state, results, workspace) fit.  A request
  that does not fit waits (it is deferred, never dropped) until retirements free memory.
* Latency is arrival -> the host seeing the completion event of the request's last step.

The device side is behind a small backend interface (``DeviceBackend``) so that the
scheduling logic can be exercised on the CPU with a fake backend.

Run: python -m paper_1903_03056_amd.serve [--requests 2000] [--rate 2000] [--seed 5]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from dataclasses import dataclass, field

import numpy as np

MASS_POOL = (1.0, 2.0, 4.0, 20.0)
N_CHOICES = (16, 24, 32, 48)
L_BOX, OMEGA, M_DESIGN = 6.0, 0.74, 12
WS_NODES = 64          # workspace of a pool covers at most this many nodes per pass


@dataclass
class Request:
    rid: int
    t_arrive: float          # seconds after the start of the trace
    masses: tuple            # ascending
    N: int
    steps: int = 50
    dt: float = 0.01
    seed: int = 5
    # filled in by the server
    t_admit: float = math.nan
    t_done: float = math.nan
    final: np.ndarray | None = field(default=None, repr=False)

    @property
    def key(self):
        return (self.N, self.masses, self.dt)

    @property
    def pair_evals(self) -> int:
        return len(self.masses) ** 2 * self.steps


def make_trace(n_requests=2000, rate=2000.0, seed=5, steps=50, dt=0.01, Ns=N_CHOICES, mass_pool=MASS_POOL):
    """Poisson arrivals (exponential gaps of mean 1/rate); 2 or 3 species per request with
    masses drawn without replacement from mass_pool; N drawn uniformly from Ns."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(n_requests):
        t += rng.exponential(1.0 / rate)
        s = int(rng.integers(2, 4))
        masses = tuple(sorted(float(m) for m in rng.choice(mass_pool, size=s, replace=False)))
        N = int(rng.choice(Ns))
        out.append(Request(rid=rid, t_arrive=t, masses=masses, N=N, steps=steps, dt=dt, seed=seed))
    return out


def initial_state(req: Request) -> np.ndarray:
    """Seeded two-Maxwellian initial data of one request, [s][N][N][N] float32."""
    from synth import inputs as I
    return I.draw_request_state(req.seed, req.rid, req.masses, req.N, L_BOX).astype(np.float32)


def state_bytes(N: int, s: int) -> int:
    """Device bytes of one slot: FP32 state f and FP32 collision result Q."""
    return 2 * 4 * s * N ** 3


class Budget:
    """Byte counter behind admission control."""

    def __init__(self, limit_bytes: int):
        self.limit = int(limit_bytes)
        self.used = 0
        self.peak = 0

    def try_take(self, nbytes: int) -> bool:
        if self.used + nbytes > self.limit:
            return False
        self.used += nbytes
        self.peak = max(self.peak, self.used)
        return True

    def give(self, nbytes: int) -> None:
        self.used -= nbytes
        if self.used < 0:
            raise RuntimeError("budget released more than it held")


def grown_capacity(cap: int, need: int) -> int:
    """Capacity after growth: doubling from 4."""
    cap = max(4, cap)
    while cap < need:
        cap *= 2
    return cap


# Gain geometry per grid size when the backend is given none.  At N = 32 the serving loop
# takes the FFT geometry (2, 1) rather than the matrix-core default: the matrix-core kernel
# holds a whole CU's LDS, so with several pools' kernels in flight it waits longer for
# CUs.  On a 500-request overload trace: 88-92 req/s against 84-88, p99 5.3-5.5 s against
# 5.6-5.8 s (two runs each).
SERVE_TILES = {32: (2, 1)}


class DeviceBackend:
    """Pools of device-resident slots on the HIP device (torch memory, libdgfs kernels)."""

    def __init__(self, tile=None, scheme: str = "euler"):
        import torch
        if scheme not in ("euler", "ssprk2"):
            raise ValueError("scheme is 'euler' or 'ssprk2'")
        self.torch = torch
        self.tile = tile
        self.scheme = scheme
        self.plans = {}

    def plan(self, key):
        from .collision import CollisionPlan
        if key not in self.plans:
            N, masses, _ = key
            tile = self.tile if self.tile is not None else SERVE_TILES.get(N)
            self.plans[key] = CollisionPlan(masses, N, L_BOX, M_DESIGN, N // 2, omega=OMEGA, precision="f32",
                                            tile=tile)
        return self.plans[key]

    def new_pool(self, key):
        return DevicePool(self, key)

    def stage(self, payload: np.ndarray):
        """Host copy of a request's initial data in pinned memory (made before it is sent)."""
        return self.torch.from_numpy(payload).pin_memory()


class DevicePool:
    def __init__(self, backend: DeviceBackend, key):
        self.torch = backend.torch
        self.plan = backend.plan(key)
        self.scheme = backend.scheme
        self.dt = key[2]
        self.s, self.N = self.plan.s, self.plan.N
        self.stream = self.torch.cuda.Stream()
        self.event = None
        self.f = self.Q = self.ws = None
        self.cap = 0
        self.peak_cap = 0          # largest slot capacity the pool has held
        self._staged = []          # pinned host buffers whose copies are in flight

    def _ws_bytes(self, cap: int) -> int:
        """Collide workspace for WS_NODES nodes per pass; SSP-RK2 adds its two stage states."""
        ws = self.plan.workspace_bytes(min(cap, WS_NODES))
        if self.scheme == "ssprk2":
            ws += 2 * (((cap * self.s * self.N ** 3 * 4) + 255) // 256 * 256)
        return ws

    def bytes_for(self, cap: int) -> int:
        if cap == 0:
            return 0
        return cap * state_bytes(self.N, self.s) + self._ws_bytes(cap)

    def resize(self, cap: int, live: int) -> None:
        torch = self.torch
        if cap == 0:
            self.f = self.Q = self.ws = None
            self.cap = 0
            return
        with torch.cuda.stream(self.stream):
            shape = (cap, self.s, self.N, self.N, self.N)
            f = torch.empty(shape, dtype=torch.float32, device="cuda")
            if live:
                f[:live].copy_(self.f[:live])
            self.f = f
            self.Q = torch.empty(shape, dtype=torch.float32, device="cuda")
            self.ws = torch.empty(self._ws_bytes(cap), dtype=torch.uint8, device="cuda")
        self.cap = cap
        self.peak_cap = max(self.peak_cap, cap)

    def insert(self, slot: int, staged) -> None:
        with self.torch.cuda.stream(self.stream):
            self.f[slot].copy_(staged, non_blocking=True)
        self._staged.append(staged)

    def move(self, dst: int, src: int) -> None:
        with self.torch.cuda.stream(self.stream):
            self.f[dst].copy_(self.f[src])

    def read(self, slot: int) -> np.ndarray:
        with self.torch.cuda.stream(self.stream):
            out = self.f[slot].cpu().numpy().copy()
        return out

    def launch(self, n: int) -> None:
        """One step (forward Euler, or SSP-RK2 through dgfs_relax) of slots [0, n) on this
        pool's stream; an event marks its end."""
        f, Q = self.f[:n], self.Q[:n]
        if self.scheme == "ssprk2":
            self.plan.relax(f, self.dt, 1, scheme="ssprk2", workspace=self.ws, stream=self.stream)
        else:
            self.plan.collide(f, out=Q, workspace=self.ws, stream=self.stream)
            self.plan.relax_step(f, Q, self.dt, stream=self.stream)
        self.event = self.torch.cuda.Event()
        self.event.record(self.stream)

    def ready(self) -> bool:
        if self.event is None or self.event.query():
            self._staged.clear()
            return True
        return False

    def sync(self) -> None:
        self.stream.synchronize()
        self._staged.clear()


class Pool:
    """Host bookkeeping of one pool: which request sits in which slot."""

    def __init__(self, key, dev):
        self.key, self.dev = key, dev
        self.slots = []            # request ids, slot order
        self.done = []             # steps completed per slot
        self.waiting = []          # admitted, not yet in a slot: (rid, staged payload)
        self.inflight = 0          # slots covered by the step in flight (0 = idle)
        self.held = 0              # bytes charged to the budget
        self.launches = 0


class Server:
    def __init__(self, backend=None, budget_bytes=None, keep_final=False, tile=None, scheme="euler"):
        if backend is None:
            backend = DeviceBackend(tile=tile, scheme=scheme)
        if budget_bytes is None:
            import torch
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(0.8 * free)
        self.backend = backend
        self.budget = Budget(budget_bytes)
        self.pools = {}
        self.keep_final = keep_final
        self.deferrals = 0

    def pool(self, key) -> Pool:
        if key not in self.pools:
            self.pools[key] = Pool(key, self.backend.new_pool(key))
        return self.pools[key]

    def warm(self, trace):
        """Build the plans and stage the initial data of every request before the clock
        starts (a client sends its data with the request)."""
        t0 = time.perf_counter()
        for key in sorted({r.key for r in trace}):
            self.pool(key)
        staged = {r.rid: self.backend.stage(initial_state(r)) for r in trace}
        return staged, time.perf_counter() - t0

    # -- admission -------------------------------------------------------------------
    def try_admit(self, req: Request, staged) -> bool:
        """Reserve the bytes the request's pool will hold with one more slot."""
        pool = self.pool(req.key)
        need = len(pool.slots) + len(pool.waiting) + 1
        target = pool.held
        if need > pool.dev.cap:
            target = max(pool.held, pool.dev.bytes_for(grown_capacity(pool.dev.cap, need)))
        if target > pool.held:
            if not self.budget.try_take(target - pool.held):
                return False
            pool.held = target
        pool.waiting.append((req.rid, staged))
        return True

    # -- one pool between steps ---------------------------------------------------------
    def _service(self, pool: Pool, reqs, clock) -> int:
        """Retire finished requests, seat waiting ones, launch the next step.  Returns
        the number of requests retired."""
        retired = 0
        if pool.inflight:
            t = clock()
            for k in range(pool.inflight):
                pool.done[k] += 1
            slot = 0
            n_live = len(pool.slots)
            while slot < n_live:
                r = reqs[pool.slots[slot]]
                if pool.done[slot] >= r.steps:
                    r.t_done = t
                    if self.keep_final:
                        r.final = pool.dev.read(slot)
                    last = n_live - 1
                    if slot != last:
                        pool.dev.move(slot, last)
                        pool.slots[slot] = pool.slots[last]
                        pool.done[slot] = pool.done[last]
                    pool.slots.pop()
                    pool.done.pop()
                    n_live -= 1
                    retired += 1
                else:
                    slot += 1
            pool.inflight = 0
        if pool.waiting:
            need = len(pool.slots) + len(pool.waiting)
            if need > pool.dev.cap:
                pool.dev.resize(grown_capacity(pool.dev.cap, need), len(pool.slots))
            for rid, staged in pool.waiting:
                pool.dev.insert(len(pool.slots), staged)
                pool.slots.append(rid)
                pool.done.append(0)
            pool.waiting.clear()
            # retirements since the reservation may leave part of it unused
            actual = pool.dev.bytes_for(pool.dev.cap)
            if actual < pool.held:
                self.budget.give(pool.held - actual)
                pool.held = actual
        if pool.slots:
            pool.dev.launch(len(pool.slots))
            pool.inflight = len(pool.slots)
            pool.launches += 1
        elif pool.held:
            pool.dev.resize(0, 0)
            self.budget.give(pool.held)
            pool.held = 0
        return retired

    def run(self, trace, staged=None, realtime=True, progress=None):
        """Serve the trace; returns the summary dict.  realtime=False admits every request
        at t=0 (arrival times ignored for admission, kept for latency)."""
        if staged is None:
            staged, _ = self.warm(trace)
        reqs = {r.rid: r for r in trace}
        order = sorted(trace, key=lambda r: r.t_arrive)
        nxt = done = 0
        t0 = time.perf_counter()

        def clock():
            return time.perf_counter() - t0

        last_report = 0
        while done < len(trace):
            now = clock() if realtime else math.inf
            while nxt < len(order) and order[nxt].t_arrive <= now:
                r = order[nxt]
                if not self.try_admit(r, staged[r.rid]):
                    self.deferrals += 1
                    break
                r.t_admit = clock()
                nxt += 1
            busy = False
            for pool in self.pools.values():
                if pool.inflight or pool.waiting:
                    busy = True
                    if pool.dev.ready():
                        done += self._service(pool, reqs, clock)
            if progress and done - last_report >= max(1, len(trace) // 10):
                last_report = done
                progress(f"{done}/{len(trace)} requests done at {clock():.1f} s")
            if busy:
                time.sleep(20e-6)
            elif nxt < len(order):
                # nothing on the device: every pool is empty and has returned its bytes
                if order[nxt].t_arrive <= (clock() if realtime else math.inf):
                    raise RuntimeError(f"request {order[nxt].rid} does not fit the HBM budget even alone")
                time.sleep(max(0.0, min(order[nxt].t_arrive - clock(), 0.005)))
        for pool in self.pools.values():
            pool.dev.sync()
        makespan = clock()
        lat = np.array([r.t_done - r.t_arrive for r in trace])
        evals = sum(r.pair_evals for r in trace)
        return {
            "requests": len(trace), "makespan_s": makespan,
            "throughput_req_s": len(trace) / makespan,
            "pair_evals_per_s": evals / makespan,
            "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)),
            "latency_max_s": float(lat.max()),
            "pools": len(self.pools), "launches": sum(p.launches for p in self.pools.values()),
            "budget_bytes": self.budget.limit, "budget_peak_bytes": self.budget.peak,
            "deferrals": self.deferrals,
        }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--budget-gb", type=float, default=None)
    ap.add_argument("--scheme", choices=["euler", "ssprk2"], default="euler",
                    help="time step of every request: forward Euler or SSP-RK2 (Sec. 5)")
    ap.add_argument("--relaxed", action="store_true",
                    help="after the trace, serve a second one at 0.7x the measured capacity")
    args = ap.parse_args()

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    budget = int(args.budget_gb * (1 << 30)) if args.budget_gb else None
    results = []
    trace = make_trace(args.requests, args.rate, args.seed, args.steps)
    srv = Server(budget_bytes=budget, scheme=args.scheme)
    staged, setup = srv.warm(trace)
    log(f"{len(srv.pools)} plans built and {len(trace)} requests staged in {setup:.1f} s")
    res = srv.run(trace, staged, progress=log)
    res.update({"rate_req_s": args.rate, "setup_s": setup})
    results.append(res)
    log(json.dumps(res))
    if args.relaxed:
        rate = 0.7 * res["throughput_req_s"]
        n = max(20, int(round(rate * 10)))
        trace2 = make_trace(n, rate, args.seed + 1, args.steps)
        srv2 = Server(backend=srv.backend, budget_bytes=budget)
        staged2, setup2 = srv2.warm(trace2)
        res2 = srv2.run(trace2, staged2, progress=log)
        res2.update({"rate_req_s": rate, "setup_s": setup2})
        results.append(res2)
        log(json.dumps(res2))
    print(json.dumps({
        "workload": "Poisson arrivals; 2-3 species with masses from {1,2,4,20}; N in {16,24,32,48}; "
                    "L=6, M=12, N_rho=N/2, VHS omega=0.74; " + ("forward Euler" if args.scheme == "euler" else "SSP-RK2")
                    + " dt=0.01 with the FP64 projection",
        "steps_per_request": args.steps, "dtype": "f32 (FP64 projection)", "runs": results}), flush=True)


if __name__ == "__main__":
    main()
