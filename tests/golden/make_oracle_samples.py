"""Sampled FP64 oracle results at the full-size workloads, for the GPU parity tests.

The oracle needs seconds to a minute per node at these sizes (N = 32 and 48, up to
576 (rho, sigma) convolutions per ordered pair), too long to run inside a GPU test for
the 16 nodes or so each workload is checked on.  This script evaluates them once, on the
host, and stores for every checked node:

* ``fsum``   [n][s]        sum of the FP32-rounded input field of each species (a
                           fingerprint: the test recomputes it from the same seeded draw);
* ``qmax``   [n][s]        max_v |Q^i| over the whole grid (Q^i = sum_j Q^{ij});
* ``qpmax``  [n][s][s]     max_v |Q^{ij}| over the whole grid;
* ``loss``   [n][s][s]     max_v |f^i nu^{ij}|, the loss term of the pair (the scale of
                           FP32 rounding where Q^{ij} itself is a small difference);
* ``idx``    [n][s][K]     flat grid indices sampled on species i's grid: the largest
                           |Q^i| and |Q^{ij}| points and a seeded uniform sample;
* ``qp``     [n][s][s][K]  Q^{ij} at those indices (summing over j gives Q^i there).

Serving trajectories store the same fields for the final state of each request
(``fsum`` of the initial state, ``qmax`` = max |f^i|, ``qp`` = f^i at the samples).

``oracle_krook_wu_N64.npz``: the Krook-Wu solution (Sec. 6.1, m1 = m2 = 1, L = 12, M = 6)
at N = 64 advanced from t = 5.5 by two SSP-RK2 steps of dt = 0.01 with N_rho = 64 (the
settings of the paper's time-evolution figure), the projected operator of the oracle;
the final state f and its change f - f0 are stored at 4096 seeded grid points per species
(with the largest |f - f0| point) beside their maxima over the whole grid.

``oracle_slab_transport_min.json``: the DG slab of 64 elements x 4 GLL nodes between
diffuse walls (N = 32, the noise-free slab inputs), advanced by transport alone with
SSP-RK2 at dt = 2e-4; min f / max f_0 after each of 20 steps.

Inputs are the seeded draws of ``synth.inputs`` rounded to FP32 (what the device
receives); the arithmetic is the oracle's, in FP64.  Nothing here touches the library.

Usage: python tests/golden/make_oracle_samples.py [--jobs 8] [--only NAME ...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

# one FFT thread per worker process: the transforms are small, processes scale better
os.environ.setdefault("OMP_NUM_THREADS", "1")

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

K_UNIFORM = 448      # uniformly drawn sample points per (node, species)
K_TOP = 60           # largest |Q^i| points per (node, species)
SAMPLE_SEED = 20190307

ARKR_MASSES = (1.0, 139.1 / 66.3)
ARKR_OMEGA = ((0.81, 0.805), (0.805, 0.8))
ARKR_ALPHA = ((1.4, 1.36), (1.36, 1.32))

# serving requests checked against the oracle trajectory (the serving test builds the
# same requests): a pool of 70 N = 32 requests (more than one 64-node workspace pass)
# and N = 48 requests
SERVE = dict(seed=55, dt=0.01, L=6.0, M=12, omega=0.74)
SERVE_TRAJ = (
    dict(rid=69, masses=(1.0, 2.0), N=32, steps=3),
    dict(rid=101, masses=(1.0, 20.0), N=48, steps=2),
)


def spread(n_total: int, n_pick: int) -> list:
    """n_pick node indices spread over [0, n_total), with consecutive picks landing on
    different residues modulo 8 (the gain kernel deals a node's workgroups to XCD
    node mod 8), the last node always included."""
    step = max(1, n_total // n_pick)
    nodes = [min(n_total - 1, k * step + (k % 8)) for k in range(n_pick - 1)]
    nodes.append(n_total - 1)
    return sorted(set(nodes))


# ------------------------------------------------------------------ workloads
def workloads():
    from synth import inputs as I
    c2, c3, c4 = I.config(2), I.config(3), I.config(4)
    out = {
        "slab_N32": dict(kind="common", seed=c2["seed"], batch=c2["batch"], masses=c2["masses"], N=c2["N"],
                         L=c2["L"], M=c2["M"], nrho=c2["nrho"], omega=c2["omega"], noise=c2["noise"],
                         nodes=spread(c2["batch"], 16)),
        "heavy_light_N48": dict(kind="species_grids", seed=c3["seed"], batch=c3["batch"], masses=c3["masses"],
                                N=c3["N"], L=c3["L"], M=c3["M"], nrho=c3["nrho"], omega=c3["omega"],
                                nodes=spread(c3["batch"], 16)),
        "vss_slab_N32": dict(kind="vss", seed=2, batch=256, masses=ARKR_MASSES, N=32, L=6.0, M=12, nrho=16,
                             noise=1e-2, nodes=spread(256, 8)),
        "serve_traj": dict(kind="serve", requests=SERVE_TRAJ, **SERVE),
    }
    for k, (N, B) in enumerate(c4["groups"]):
        out[f"uneven_N{N}"] = dict(kind="uneven", cls=k, seed=c4["seed"], groups=c4["groups"], masses=c4["masses"],
                                   N=N, L=c4["L"], M=c4["M"], nrho=N // 2, omega=c4["omega"],
                                   nodes=spread(B, 8 if N < 48 else 4))
    return out


def draw_inputs(w):
    """FP32-rounded float64 inputs of the whole batch (the device's view)."""
    from synth import inputs as I
    if w["kind"] in ("common", "vss"):
        f = I.draw_bimaxwellian_batch(np.random.default_rng(w["seed"]), w["batch"], len(w["masses"]), w["N"],
                                      w["L"], w["masses"], noise=w["noise"])
    elif w["kind"] == "species_grids":
        Ls = tuple(w["L"] * np.sqrt(1.0 / m) for m in w["masses"])
        f = I.draw_config3_batch(np.random.default_rng(w["seed"]), w["batch"], w["N"], Ls, w["masses"])
    elif w["kind"] == "uneven":
        f = I.draw_uneven_groups(w["seed"], w["groups"], len(w["masses"]), w["L"], w["masses"])[w["cls"]]
    else:
        raise ValueError(w["kind"])
    return f.astype(np.float32).astype(np.float64)


def problem(w):
    from oracle import params as OP, spectral as OS
    if w["kind"] == "vss":
        s = len(w["masses"])
        kern = [[(ARKR_OMEGA[i][j], ARKR_ALPHA[i][j],
                  OP.vss_prefactor(w["masses"][i], w["masses"][j], ARKR_OMEGA[i][j], ARKR_ALPHA[i][j]))
                 for j in range(s)] for i in range(s)]
        return OS.Problem(masses=tuple(w["masses"]), L=w["L"], N=w["N"], M=w["M"], nrho=w["nrho"], kernel=kern)
    return OS.vhs_problem(w["masses"], w["omega"], w["L"], w["N"], w["M"], w["nrho"])


def grids_of(w):
    if w["kind"] == "species_grids":
        return tuple(w["L"] * np.sqrt(1.0 / m) for m in w["masses"])
    return (w["L"],) * len(w["masses"])


# ------------------------------------------------------------------- oracle
def loss_terms(f, prob, Ls):
    """max_v |f^i nu^{ij}| per ordered pair, on species i's grid."""
    from oracle import grids as OG, spectral as OS
    s, N = prob.s, f.shape[-1]
    KX, KY, KZ = OS.mode_grids(N)
    kabs = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    out = np.zeros((s, s))
    for i in range(s):
        for j in range(s):
            Lij = max(Ls[i], Ls[j])
            fi = f[i] if Ls[i] == Lij else OG.interpolate(f[i], Ls[i], Lij)
            fj = f[j] if Ls[j] == Lij else OG.interpolate(f[j], Ls[j], Lij)
            om, al, C = prob.kernel[i][j]
            pr = OS.make_pair(prob.masses[i], prob.masses[j], om, C, Lij, prob.nrho, prob.sigma, prob.wsigma,
                              alpha=al)
            fhi, fhj = OS._coefficients_fft(fi), OS._coefficients_fft(fj)
            loss = OS._synthesize_fft(OS.circular_convolution(fhi, pr.loss(kabs) * fhj)).real
            if Ls[i] != Lij:
                loss = OG.interpolate(loss, Lij, Ls[i])
            out[i, j] = np.abs(loss).max()
    return out


def sample_indices(Qi_sum, Qi_pairs, rng):
    """K_TOP largest |Q^i| points, the argmax of each |Q^{ij}|, then uniform points (no
    repeats), K_UNIFORM + K_TOP + s values in all (padded with uniform draws)."""
    n = Qi_sum.size
    top = np.argsort(np.abs(Qi_sum).ravel())[::-1][:K_TOP]
    picks = list(top) + [int(np.argmax(np.abs(q))) for q in Qi_pairs]
    seen = set(int(p) for p in picks)
    want = K_UNIFORM + K_TOP + len(Qi_pairs)
    out = [int(p) for p in dict.fromkeys(picks)]
    while len(out) < want:
        p = int(rng.integers(0, n))
        if p not in seen:
            seen.add(p)
            out.append(p)
    return np.array(out[:want], dtype=np.int64)


def node_record(name, w, b, f):
    """Oracle record of node b (f: its FP32-rounded input [s][N][N][N])."""
    from oracle import grids as OG, spectral as OS
    t0 = time.time()
    prob = problem(w)
    Ls = grids_of(w)
    if w["kind"] == "species_grids":
        Qp = OG.collide_pairs(f, prob, Ls)
    else:
        Qp = OS.collide_pairs(f, prob)
    s = prob.s
    Q = Qp.sum(axis=1)
    rng = np.random.default_rng([SAMPLE_SEED, b])
    idx = np.stack([sample_indices(Q[i], [Qp[i, j] for j in range(s)], rng) for i in range(s)])
    rec = dict(node=b, fsum=f.reshape(s, -1).sum(axis=1),
               qmax=np.abs(Q).reshape(s, -1).max(axis=1),
               qpmax=np.abs(Qp).reshape(s, s, -1).max(axis=2),
               loss=loss_terms(f, prob, Ls),
               idx=idx,
               qp=np.stack([np.stack([Qp[i, j].ravel()[idx[i]] for j in range(s)]) for i in range(s)]))
    print(f"{name}: node {b} done in {time.time() - t0:.1f} s", flush=True)
    return rec


def serve_record(w, req):
    """The oracle's Euler trajectory of one request: f <- f + dt P(Q(f)), P the FP64
    projection, from the FP32-rounded initial state."""
    from oracle import moments as OM, spectral as OS
    from synth import inputs as I
    t0 = time.time()
    masses, N = tuple(req["masses"]), req["N"]
    s = len(masses)
    f0 = I.draw_request_state(w["seed"], req["rid"], masses, N, w["L"]).astype(np.float32).astype(np.float64)
    prob = OS.vhs_problem(masses, w["omega"], w["L"], N, w["M"], N // 2)
    f = f0.copy()
    for _ in range(req["steps"]):
        f = f + w["dt"] * OM.conserve(OS.collide(f, prob), masses, (w["L"],) * s)
    rng = np.random.default_rng([SAMPLE_SEED, req["rid"]])
    idx = np.stack([sample_indices(f[i], [f[i]], rng) for i in range(s)])
    rec = dict(node=req["rid"], fsum=f0.reshape(s, -1).sum(axis=1), qmax=np.abs(f).reshape(s, -1).max(axis=1),
               idx=idx, qp=np.stack([f[i].ravel()[idx[i]][None] for i in range(s)]))
    print(f"serve_traj: request {req['rid']} done in {time.time() - t0:.1f} s", flush=True)
    return rec


_SELECTED = {}


def selected_inputs(name, w):
    """The checked nodes' inputs of workload ``name`` (drawn once per process)."""
    if name not in _SELECTED:
        if w["kind"] == "species_grids":
            # node by node from one generator: the same draws as one call for the whole
            # batch (no batch-wide noise), without holding the batch in memory
            from synth import inputs as I
            Ls = grids_of(w)
            rng = np.random.default_rng(w["seed"])
            sel = {}
            for b in range(max(w["nodes"]) + 1):
                f = I.draw_config3_batch(rng, 1, w["N"], Ls, w["masses"])[0]
                if b in w["nodes"]:
                    sel[b] = f.astype(np.float32).astype(np.float64)
            _SELECTED[name] = sel
        else:
            f = draw_inputs(w)
            _SELECTED[name] = {b: f[b].copy() for b in w["nodes"]}
    return _SELECTED[name]


def slab_transport_minima(steps=20, dt=2e-4):
    """min f / max f_0 after each SSP-RK2 step of the oracle's DG transport (Sec. 5, no
    collision term) on the slab workload's noise-free inputs."""
    from oracle import dg, stepping as T
    from synth import inputs as I
    c = I.config(2)
    Ne, K, N, L, masses = 64, 4, c["N"], c["L"], c["masses"]
    slab = dg.Slab(0.0, 1.0, Ne, K, masses, N, (L, L), dg.Boundary("wall", u=(0.0, -0.3, 0.0), T=1.0),
                   dg.Boundary("wall", u=(0.0, 0.3, 0.0), T=1.0))
    f = I.draw_bimaxwellian_batch(np.random.default_rng(c["seed"]), Ne * K, 2, N, (L, L), masses)
    F = f.astype(np.float32).astype(np.float64).reshape(Ne, K, 2, N, N, N)
    top = F.max()
    lows = []
    for _ in range(steps):
        F = T.ssprk2(F, slab.transport, dt, 1)
        lows.append(float(F.min() / top))
    path = os.path.join(HERE, "oracle_slab_transport_min.json")
    with open(path, "w") as fh:
        json.dump({"what": "min f / max f0 after each SSP-RK2 step, DG transport only (Sec. 5), 64 x 4 GLL "
                           "nodes on [0, 1], diffuse walls u_y = -+0.3, T = 1, N = 32, L = 6, masses (1, 2), "
                           "noise-free bi-Maxwellians (seed 2), dt = 2e-4",
                   "dt": dt, "min_over_max0": lows}, fh, indent=1)
    print(f"wrote {path}", flush=True)


def _pair_task(args):
    from oracle import spectral as OS
    f, prob, i, j = args
    return i, j, OS.collide_pair_fast(f[i], f[j], prob.pair(i, j))


def krook_wu_N64(jobs, steps=2, dt=0.01, t0=5.5):
    """Two SSP-RK2 steps of the Krook-Wu data at N = 64, N_rho = 64, with the four ordered
    pairs of every stage evaluated in parallel processes."""
    import multiprocessing as mp

    from oracle import bkw, moments as OM, spectral as OS
    kw = bkw.KrookWu(1.0, 1.0)
    N, L, M, nrho = 64, 12.0, 6, 64
    kern = [[(1.0, 1.0, kw.kernel_constant(i + 1, j + 1)) for j in range(2)] for i in range(2)]
    prob = OS.Problem(masses=kw.m, L=L, N=N, M=M, nrho=nrho, kernel=kern)
    f0, _ = kw.on_grid(N, L, t0)
    t_start = time.time()
    with mp.get_context("spawn").Pool(min(jobs, 4)) as pool:
        def rhs(f):
            Q = np.zeros_like(f)
            for i, j, q in pool.map(_pair_task, [(f, prob, i, j) for i in range(2) for j in range(2)]):
                Q[i] += q
            return OM.conserve(Q, kw.m, (L, L))
        f = f0.copy()
        for _ in range(steps):
            f1 = f + dt * rhs(f)
            f = 0.5 * f + 0.5 * (f1 + dt * rhs(f1))
    fe, _ = kw.on_grid(N, L, t0 + steps * dt)
    d = (f - f0).reshape(2, -1)
    rng = np.random.default_rng([SAMPLE_SEED, 64])
    idx = np.stack([np.concatenate([[int(np.argmax(np.abs(d[i])))], rng.integers(0, N ** 3, size=4095)])
                    for i in range(2)])
    fr = f.reshape(2, -1)
    path = os.path.join(HERE, "oracle_krook_wu_N64.npz")
    meta = dict(ratio=1.0, N=N, L=L, M=M, nrho=nrho, dt=dt, steps=steps, t0=t0, scheme="ssprk2")
    np.savez_compressed(path, idx=idx, f=np.stack([fr[i, idx[i]] for i in range(2)]),
                        df=np.stack([d[i, idx[i]] for i in range(2)]), fmax=np.abs(fr).max(axis=1),
                        dfmax=np.abs(d).max(axis=1), meta=np.array(json.dumps(meta)))
    print(f"wrote {path} ({time.time() - t_start:.0f} s); error vs the exact solution "
          f"{np.abs(f - fe).max():.3e}", flush=True)


def _task(args):
    name, b = args
    w = workloads()[name]
    if w["kind"] == "serve":
        return name, serve_record(w, w["requests"][b])
    return name, node_record(name, w, b, selected_inputs(name, w)[b])


def save(name, w, recs):
    meta = {k: v for k, v in w.items() if k not in ("requests",)}
    if w["kind"] == "serve":
        meta["requests"] = list(w["requests"])
    arrays = {}
    if w["kind"] == "serve":
        # requests may differ in s and N: one group of arrays per request
        for k, r in enumerate(recs):
            for key in ("fsum", "qmax", "idx", "qp"):
                arrays[f"r{k}_{key}"] = r[key]
    else:
        for key in ("fsum", "qmax", "qpmax", "loss", "idx", "qp"):
            arrays[key] = np.stack([r[key] for r in recs])
        arrays["nodes"] = np.array([r["node"] for r in recs], dtype=np.int64)
    arrays["meta"] = np.array(json.dumps(meta))
    path = os.path.join(HERE, f"oracle_{name}.npz")
    np.savez_compressed(path, **arrays)
    print(f"wrote {path} ({os.path.getsize(path) / 1024:.0f} KiB)", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", nargs="*", default=None)
    args = ap.parse_args()
    if args.only is None or "slab_transport_min" in args.only:
        slab_transport_minima()
    if args.only is None or "krook_wu_N64" in args.only:
        krook_wu_N64(args.jobs)
    ws = workloads()
    names = [n for n in ws if args.only is None or n in args.only]
    tasks = []
    for n in names:
        count = len(ws[n]["requests"]) if ws[n]["kind"] == "serve" else len(ws[n]["nodes"])
        tasks += [(n, k if ws[n]["kind"] == "serve" else ws[n]["nodes"][k]) for k in range(count)]
    # the longest tasks first
    cost = {"heavy_light_N48": 60, "uneven_N48": 70, "serve_traj": 60, "vss_slab_N32": 12, "slab_N32": 7,
            "uneven_N32": 15, "uneven_N24": 6}
    tasks.sort(key=lambda t: -cost.get(t[0], 1))
    results = {n: [] for n in names}
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(args.jobs) as pool:
        for name, rec in pool.imap_unordered(_task, tasks):
            results[name].append(rec)
            w = ws[name]
            total = len(w["requests"]) if w["kind"] == "serve" else len(w["nodes"])
            if len(results[name]) == total:
                recs = sorted(results[name], key=lambda r: r["node"])
                save(name, w, recs)


if __name__ == "__main__":
    main()
