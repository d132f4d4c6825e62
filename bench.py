"""Benchmark of the batched multi-species collision operator on one MI355X.

Workload (one "step"): the 1-D DG slab of 64 elements x 4 GLL nodes = 256 independent
spatial points, 2 species with masses (1, 2), VHS omega = 0.74, N = 32, L = 6, M = 12
(icosahedron), N_rho = 16, seeded bi-Maxwellians with 1e-2 uniform noise.  A step is
the whole hot path: forward transforms, gain (rho, sigma) loop, radial sum and loss,
inverse transforms and combination (dgfs_collide), then the FP64 conservation
projection (dgfs_conserve).  Inputs are resident in device memory before timing.

Also measured, outside the timed steps (the "workloads" object):
  * uneven batch: 512 nodes at N=24, 256 at N=32 and 64 at N=48, 3 species (1, 2, 4),
    N_rho = N/2, autotuned gain-kernel tiles, the whole batch captured once in a hipGraph
    and replayed (per-replay p50/p99);
  * heavy/light species-specific grids: 1024 nodes, masses (1, 32.75) on boxes
    L_i = 6 sqrt(1/m_i), hard spheres, N=48, M=24 (7-design), N_rho=24;
  * VSS kernels: the slab shape with the argon-krypton VSS parameters (sigma-dependent
    kernel mode, one transform per direction);
  * SSP-RK2 time stepping of the slab (two projected operator evaluations per step);
  * the slab as a DG solver: nodal DG transport between two diffuse walls plus the
    projected collisions, SSP-RK2;
  * the slab with eq. (sum) as a linear (dealiased) convolution, padded to 3N/2;
  * measured ceilings: a device copy (HBM) and an FMA loop (FP32 vector).

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = dict(batch=256, masses=(1.0, 2.0), omega=0.74, N=32, L=6.0, M=12, n_rho=16, noise=1e-2, seed=2)
PEAK_FP32_VECTOR_TFLOPS = 157.3   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz
PEAK_HBM_GBPS = 8000.0
PEAK_FP16_MFMA_TFLOPS = 2500.0    # dense FP16 matrix cores


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gain_flops_per_node(N, M, n_rho, s, antipodal=True):
    """Algorithmic flops of the gain stage for one node (the work the chosen algorithm
    must do): per gain class, direction and radial point two inverse 3-D FFTs of the
    phase-shifted spectra (5 N^3 log2 N^3 each) plus the phase product (6 flops per
    point per field) and the product-accumulate (10 flops per point); per class and
    radial point one forward 3-D FFT.  With an antipodal design the two orderings of an
    unlike pair share one class and a like pair needs M/2 directions."""
    n3 = N ** 3
    fft = 5.0 * n3 * math.log2(n3)
    if antipodal:
        dirs = s * (M // 2) + (s * (s - 1) // 2) * M
        ncls = s + s * (s - 1) // 2
    else:
        dirs = s * s * M
        ncls = s * s
    return dirs * n_rho * (2 * (fft + 6 * n3) + 10 * n3) + ncls * n_rho * fft


def gain_flops_per_node_vss(N, M, n_rho, s, antipodal=True):
    """The same for a VSS kernel, whose kernel mode depends on the direction: per
    direction and radial point two inverse 3-D FFTs with their phase products, the
    complex product (12 flops per point) and one forward 3-D FFT (the library transforms
    the real parts of two directions together: the model counts the method's work)."""
    n3 = N ** 3
    fft = 5.0 * n3 * math.log2(n3)
    dirs = s * (M // 2) + (s * (s - 1) // 2) * M if antipodal else s * s * M
    return dirs * n_rho * (2 * (fft + 6 * n3) + 12 * n3 + fft)


def mfma_flops_per_launch(batch, N, M, n_rho, s):
    """Matrix-core flops the (2, 0) gain geometry executes per launch: per work item (node,
    class, rho_q, x-chunk) and field, the x-contraction (8 wavefronts x 8 tiles x 3 split
    products of 16x16x32), the per-wavefront C_y product of the plane vectors (6 of
    32x32x16), the two planes' z- and y-contractions (8 x 2 x 12) and the a_x plane (12);
    two fields per direction, two chunks."""
    assert N == 32
    per_field = 8 * 8 * 3 * 16384 + 8 * 6 * 32768 + 8 * 2 * 12 * 32768 + 12 * 32768
    class_dirs = s * (M // 2) + s * (s - 1) // 2 * M   # antipodal design
    return batch * class_dirs * n_rho * 2 * 2 * per_field


def load_traffic():
    """HBM bytes per launch of the gain kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source (else None)."""
    from paper_1903_03056_amd.rocprof_summary import gain_source_digest
    path = os.path.join(ROOT, "profiles", "gain_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_sha256") != gain_source_digest():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(f64, max_seconds=12.0):
    """The FP64 oracle on a bounded sample of the same workload (whole nodes, all
    ordered pairs), timed on the host cores."""
    from oracle import spectral as OS
    w = WORKLOAD
    prob = OS.vhs_problem(w["masses"], w["omega"], w["L"], w["N"], w["M"], w["n_rho"])
    t0 = time.perf_counter()
    outs, nodes = [], 0
    while nodes < f64.shape[0]:
        outs.append(OS.collide(f64[nodes], prob))
        nodes += 1
        if time.perf_counter() - t0 > max_seconds:
            break
    dt = time.perf_counter() - t0
    s = len(w["masses"])
    return {"value": nodes * s * s / dt, "unit": "evals/s", "cores": OS.WORKERS, "kind": "oracle",
            "sample": f"{nodes} of {w['batch']} nodes x {s * s} ordered pairs, FP64 numpy/scipy.fft "
                      f"({dt:.1f} s)"}, outs


def stored_oracle_errors(name, Q, summed_scale="qmax"):
    """Sampled FP64 oracle results of the nodes stored for workload `name`
    (tests/golden/oracle_<name>.npz, written from the oracle alone): max over the sampled
    points of |Q - Q_ref| per (node, species), over max_v |Q_ref| or, with
    summed_scale="loss", over the largest of the pairs' loss terms max_v |f^i nu^{ij}|.
    Q: device tensor of the whole batch.  Returns the max and median over (node, species)."""
    path = os.path.join(ROOT, "tests", "golden", f"oracle_{name}.npz")
    d = np.load(path, allow_pickle=False)
    errs = []
    for k, b in enumerate(d["nodes"]):
        q = Q[int(b)].double().cpu().numpy().reshape(d["qmax"].shape[1], -1)
        ref = d["qp"][k].sum(axis=1)
        scale = d["qmax"][k] if summed_scale == "qmax" else d["loss"][k].max(axis=1)
        errs += [float(np.abs(q[i, d["idx"][k][i]] - ref[i]).max() / scale[i]) for i in range(q.shape[0])]
    return {"nodes": len(d["nodes"]), "scale": "max|Q|" if summed_scale == "qmax" else "loss term",
            "max": max(errs), "median": float(np.median(errs))}


def measured_peaks(torch, dev):
    """A 1 GiB device copy (HBM read + write) and the library's FMA-loop probe."""
    import ctypes

    from paper_1903_03056_amd import _lib
    n = 256 * 1024 * 1024
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbps = 5 * 2 * n * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    blocks, iters = 256 * 16, 2048
    scratch = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    tf = ctypes.c_double()
    lib = _lib.load()
    _lib.check(lib.dgfs_probe_valu(ctypes.c_void_p(scratch.data_ptr()), scratch.numel() * 4, blocks, iters,
                                   ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream), ctypes.byref(tf)),
               "dgfs_probe_valu")
    return {"hbm_copy_GBps": round(copy_gbps, 1), "valu_fp32_fma_TFLOPs": round(tf.value, 2),
            "note": "copy: 5 x 1 GiB device-to-device, read+write bytes; FMA loop: unpacked FP32 FMA chains"}


def group_leg(torch, dev, replays):
    """Uneven batch of three N-classes in one hipGraph (autotuned tiles)."""
    from paper_1903_03056_amd import CollisionGroup, CollisionPlan
    from synth import inputs as I
    cfg = I.config(4)
    masses, s, L, M, omega = cfg["masses"], cfg["s"], cfg["L"], cfg["M"], cfg["omega"]
    rng = np.random.default_rng(cfg["seed"])
    plans, fs, host = [], [], []
    t0 = time.perf_counter()
    for N, B in cfg["groups"]:
        plans.append(CollisionPlan(masses, N, L, M, N // 2, omega=omega, precision="f32", tile="auto"))
        h = I.draw_bimaxwellian_batch(rng, B, s, N, L, masses).astype(np.float32)
        host.append(h)
        fs.append(torch.tensor(h, device=dev))
    setup_s = time.perf_counter() - t0
    group = CollisionGroup(plans)
    graph, outs = group.capture(fs)
    for _ in range(2):
        graph.launch()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(replays)]
    for e0, e1 in evs:
        e0.record(graph.stream)
        graph.launch()
        e1.record(graph.stream)
    torch.cuda.synchronize()
    ms = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
    evals = sum(B * s * s for _, B in cfg["groups"])
    flops = sum(B * gain_flops_per_node(N, M, N // 2, s) for N, B in cfg["groups"])
    # the same classes run one after another on one stream, each as its own collide call
    # (no overlap between classes): the sum the graph's concurrent classes compete with
    st = torch.cuda.current_stream(dev)
    for p, x, q in zip(plans, fs, outs):
        p.collide(x, out=q, workspace=p.workspace(x.shape[0], dev))
    torch.cuda.synchronize()
    iso = np.zeros((replays, len(plans)))
    for k in range(replays):
        for c, (p, x, q) in enumerate(zip(plans, fs, outs)):
            a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a0.record(st)
            p.collide(x, out=q, workspace=p.workspace(x.shape[0], dev))
            a1.record(st)
            a1.synchronize()
            iso[k, c] = a0.elapsed_time(a1)
    iso_ms = iso.mean(axis=0)
    res = {"workload": "uneven batch: 512 nodes N=24 + 256 N=32 + 64 N=48, 3 species m=(1,2,4), VHS "
                       "omega=0.74, L=6, M=12, N_rho=N/2, bi-Maxwellians, seed 4; one hipGraph replay per call",
           "value": round(evals / (ms.mean() * 1e-3), 1), "unit": "evals/s", "replays": replays,
           "ms_per_call": {"mean": round(float(ms.mean()), 3), "p50": round(float(np.percentile(ms, 50)), 3),
                           "p99": round(float(np.percentile(ms, 99)), 3)},
           "gain_tflops_over_call": round(flops / (ms.mean() * 1e-3) / 1e12, 2),
           "isolated_classes_ms": {str(N): round(float(t), 3) for (N, _), t in zip(cfg["groups"], iso_ms)},
           "isolated_sum_ms": round(float(iso_ms.sum()), 3),
           "graph_speedup_over_isolated_sum": round(float(iso_ms.sum() / ms.mean()), 4),
           "tiles": {str(p.N): list(p.tile) if p.tile else None for p in plans},
           "setup_s_incl_autotune": round(setup_s, 1),
           "rel_linf_vs_stored_oracle_samples": {str(N): stored_oracle_errors(f"uneven_N{N}", q)
                                                 for (N, _), q in zip(cfg["groups"], outs)}}
    # node 0 of the N=24 and N=32 classes, for the oracle comparison of the CPU leg
    checks = [dict(leg="uneven_group_graph", key=str(N), f=host[k][0].astype(np.float64),
                   got=outs[k][0].double().cpu().numpy(), masses=masses, omega=omega, Ls=(L,) * s, N=N, M=M,
                   nrho=N // 2) for k, (N, B) in enumerate(cfg["groups"][:2])]
    graph.close()
    group.close()
    return res, checks


def serving_leg(torch, dev, requests=500, rate=2000.0, relaxed_s=4.0):
    """The serving loop (continuous batching): Poisson arrivals at `rate` of spatially
    homogeneous relaxation problems (2-3 species with masses from {1, 2, 4, 20}, N from
    {16, 24, 32, 48}, 50 forward-Euler steps of dt = 0.01 with the FP64 projection, L = 6,
    M = 12, N_rho = N/2), then a second trace at 0.7x the throughput the first one
    measured, so latency without queueing is visible.  Latency = arrival -> completion."""
    from paper_1903_03056_amd import serve as S
    t0 = time.perf_counter()
    backend = S.DeviceBackend()
    trace = S.make_trace(requests, rate, 5, 50)
    srv = S.Server(backend=backend)
    staged, setup = srv.warm(trace)
    over = srv.run(trace, staged)
    rate2 = 0.7 * over["throughput_req_s"]
    trace2 = S.make_trace(max(20, int(round(rate2 * relaxed_s))), rate2, 6, 50)
    srv2 = S.Server(backend=backend)
    staged2, _ = srv2.warm(trace2)
    relaxed = srv2.run(trace2, staged2)
    keep = ("requests", "makespan_s", "throughput_req_s", "pair_evals_per_s", "latency_p50_s", "latency_p99_s",
            "latency_max_s", "pools", "launches", "budget_peak_bytes", "deferrals")

    def pick(r, arrival):
        out = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items() if k in keep}
        out["arrival_rate_req_s"] = round(arrival, 2)
        return out

    return {"workload": "serving: Poisson arrivals, 2-3 species with masses from {1,2,4,20}, N from {16,24,32,48}, "
                        "L=6, M=12, N_rho=N/2, VHS omega=0.74, 50 forward-Euler steps dt=0.01 with the FP64 "
                        "projection per request; continuous batching in per-(N, masses) pools, HBM-budget admission",
            "overload": pick(over, rate), "relaxed_0p7_capacity": pick(relaxed, rate2),
            "plans_and_staging_s": round(setup, 2), "leg_s": round(time.perf_counter() - t0, 1)}


def species_grid_leg(torch, dev, calls):
    """1024 heavy/light nodes on species-specific grids, N=48, M=24, N_rho=24."""
    from paper_1903_03056_amd import CollisionPlan
    from synth import inputs as I
    cfg = I.config(3)
    masses, N, M, nrho, B = cfg["masses"], cfg["N"], cfg["M"], cfg["nrho"], cfg["batch"]
    Ls = tuple(cfg["L"] * math.sqrt(1.0 / m) for m in masses)
    f = I.draw_config3_batch(np.random.default_rng(cfg["seed"]), B, N, Ls, masses).astype(np.float32)
    t0 = time.perf_counter()
    plan = CollisionPlan(masses, N, Ls, M, nrho, omega=cfg["omega"], precision="f32", tile="auto")
    setup_s = time.perf_counter() - t0
    ft = torch.tensor(f, device=dev)
    ws = torch.empty(plan.workspace_bytes(256), dtype=torch.uint8, device=dev)
    Q = torch.empty_like(ft)
    plan.collide(ft, out=Q, workspace=ws)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream(dev)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
    for e0, e1 in evs:
        e0.record(st)
        plan.collide(ft, out=Q, workspace=ws)
        e1.record(st)
    torch.cuda.synchronize()
    ms = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
    s = len(masses)
    flops = B * gain_flops_per_node(N, M, nrho, s, antipodal=False)
    res = {"workload": "heavy/light: 1024 nodes, m=(1,32.75) on species grids L=(6, 1.0484), hard spheres, "
                       "N=48, M=24 (7-design), N_rho=24, Maxwellians at rest, seed 3; 256-node workspace slices",
           "value": round(B * s * s / (ms.mean() * 1e-3), 1), "unit": "evals/s", "calls": calls,
           "ms_per_call": {"mean": round(float(ms.mean()), 2), "p50": round(float(np.percentile(ms, 50)), 2),
                           "p99": round(float(np.percentile(ms, 99)), 2)},
           "gain_tflops_over_call": round(flops / (ms.mean() * 1e-3) / 1e12, 2),
           "tile": list(plan.tile) if plan.tile else None, "setup_s_incl_autotune": round(setup_s, 1),
           # Maxwellians at rest: Q^i is a few per cent of its gain and loss terms, so both
           # measures are reported
           "rel_linf_vs_stored_oracle_samples": {"over_max_Q": stored_oracle_errors("heavy_light_N48", Q),
                                                 "over_loss_term": stored_oracle_errors("heavy_light_N48", Q,
                                                                                        "loss")}}
    # the last node (in the ragged final slice), for the oracle comparison of the CPU leg
    checks = [dict(leg="heavy_light_species_grids", key="last node", f=f[B - 1].astype(np.float64),
                   got=Q[B - 1].double().cpu().numpy(), masses=masses, omega=cfg["omega"], Ls=Ls, N=N, M=M,
                   nrho=nrho)]
    return res, checks


VSS_WORKLOAD = dict(batch=256, masses=(1.0, 139.1 / 66.3), omega=((0.81, 0.805), (0.805, 0.8)),
                    alpha=((1.4, 1.36), (1.36, 1.32)), N=32, L=6.0, M=12, n_rho=16, noise=1e-2, seed=2)


def vss_leg(torch, dev, calls):
    """The slab shape with the argon-krypton VSS kernels (sigma-dependent kernel mode),
    FP32; stage times from the timed collide."""
    from paper_1903_03056_amd import CollisionPlan, vss_kernel
    from synth import inputs as I
    w = VSS_WORKLOAD
    s = len(w["masses"])
    kern = vss_kernel(w["masses"], w["omega"], w["alpha"])
    f = I.draw_bimaxwellian_batch(np.random.default_rng(w["seed"]), w["batch"], s, w["N"], w["L"], w["masses"],
                                  noise=w["noise"]).astype(np.float32)
    t0 = time.perf_counter()
    plan = CollisionPlan(w["masses"], w["N"], w["L"], w["M"], w["n_rho"], kernel=kern, precision="f32")
    setup_s = time.perf_counter() - t0
    ft = torch.tensor(f, device=dev)
    ws = plan.workspace(w["batch"], dev)
    Q = torch.empty_like(ft)
    plan.collide(ft, out=Q, workspace=ws)
    torch.cuda.synchronize()
    stage = np.zeros(5)
    st = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(calls):
        _, ms = plan.collide_timed(ft, out=Q, workspace=ws)
        stage += np.array(ms)
    e1.record(st)
    torch.cuda.synchronize()
    ms_call = e0.elapsed_time(e1) / calls
    stage /= calls
    flops = w["batch"] * gain_flops_per_node_vss(w["N"], w["M"], w["n_rho"], s)
    # radial stage bytes: each class's (two directions) whole-spectrum partial read once
    # per node, the F_H table of each (direction, target) use once per group of 4 nodes,
    # the gain and loss spectra written, the loss terms' f_hat read (the F_A table and the
    # Nyquist-plane spectra, read only by lanes on those planes, are not counted)
    N3, NREP = w["N"] ** 3, w["N"] * w["N"] * (w["N"] // 2 + 1)
    dirs = s * (w["M"] // 2) + (s * (s - 1) // 2) * w["M"]
    uses = s * (w["M"] // 2) + s * (s - 1) * w["M"]
    radial_bytes = w["batch"] * ((dirs // 2) * w["n_rho"] * N3 * 8 + uses * w["n_rho"] * NREP * 8 / 4
                                 + 2 * s * N3 * 8 + s * s * N3 * 8)
    res = {"workload": "VSS slab: 256 nodes, argon-krypton VSS kernels (omega 0.81/0.805/0.8, alpha "
                       "1.4/1.36/1.32, m2/m1 = 2.098), N=32, L=6, M=12, N_rho=16, bi-Maxwellian + 1e-2 noise, "
                       "seed 2, FP32",
           "value": round(w["batch"] * s * s / (ms_call * 1e-3), 1), "unit": "evals/s", "calls": calls,
           "ms_per_call": round(ms_call, 3),
           "stages_ms": {"forward_fft": round(stage[0], 4), "gain": round(stage[1], 4),
                         "radial_loss": round(stage[2], 4), "inverse_xy": round(stage[3], 4),
                         "inverse_z_combine": round(stage[4], 4)},
           "gain_tflops": round(flops / (stage[1] * 1e-3) / 1e12, 2),
           "roofline": {
               "gain": {"bound": "alu", "achieved": round(flops / (stage[1] * 1e-3) / 1e12, 3),
                        "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(flops / (stage[1] * 1e-3) / 1e12 / PEAK_FP32_VECTOR_TFLOPS, 4),
                        "flop_per_launch": flops},
               "radial": {"bound": "hbm", "achieved": round(radial_bytes / (stage[2] * 1e-3) / 1e9, 1),
                          "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                          "frac": round(radial_bytes / (stage[2] * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4),
                          "bytes_per_launch": radial_bytes}},
           "setup_s": round(setup_s, 2),
           "rel_linf_vs_stored_oracle_samples": stored_oracle_errors("vss_slab_N32", Q)}
    return res


def slab_leg(torch, dev, plan, w, steps, dt=2e-4):
    """The slab workload as a DG solver (Sec. 5): 64 elements x 4 GLL nodes on [0, 1]
    between two diffuse walls moving at -+0.3 in y (T = 1), SSP-RK2: per step two
    collide calls, two transport passes and the projected updates.  dt keeps the
    transport CFL number |v_x|max dt / h = 6 x 2e-4 x 64 = 0.077 below the SSP-RK2
    limit for cubic elements with upwind flux (0.24, from the eigenvalues of the
    operator).  The initial state is the slab's bi-Maxwellians without the noise floor
    (a floor over the whole box is a hot tail the walls would re-emit as slow
    particles)."""
    from paper_1903_03056_amd import Slab, slab_gll
    from synth import inputs as I
    s = len(w["masses"])
    f32 = I.draw_bimaxwellian_batch(np.random.default_rng(w["seed"]), w["batch"], s, w["N"], w["L"],
                                    w["masses"]).astype(np.float32)
    xi, wq = slab_gll(4)
    hv3 = (2 * w["L"] / w["N"]) ** 3
    wt = torch.tensor(np.tile(wq, 64) / 64 / 2 * hv3, dtype=torch.float64, device=dev)

    def mass(f):
        return (f.double().sum(dim=(2, 3, 4)) * wt[:, None]).sum(dim=0).cpu().numpy()

    slab = Slab(plan, 0.0, 1.0, 64, 4, dict(kind="wall", u=(0.0, -0.3, 0.0), T=1.0),
                dict(kind="wall", u=(0.0, 0.3, 0.0), T=1.0))
    f = torch.tensor(f32, device=dev)
    ws = torch.empty(slab.workspace_bytes(), dtype=torch.uint8, device=dev)
    m0 = mass(f)
    slab.step(f, dt, 1, workspace=ws)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    slab.step(f, dt, steps, workspace=ws)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    m1 = mass(f)
    ok = bool(torch.isfinite(f).all())
    slab.close()
    # transport alone (collisions off): per SSP-RK2 step two transport passes (each reads
    # the state plus two face traces per element and writes the stage state), two wall
    # reductions and the averaging pass (two reads, one write)
    tslab = Slab(plan, 0.0, 1.0, 64, 4, dict(kind="wall", u=(0.0, -0.3, 0.0), T=1.0),
                 dict(kind="wall", u=(0.0, 0.3, 0.0), T=1.0), collide=False)
    tws = torch.empty(tslab.workspace_bytes(), dtype=torch.uint8, device=dev)
    tslab.step(f, dt, 1, workspace=tws)
    e0.record(st)
    tslab.step(f, dt, 20, workspace=tws)
    e1.record(st)
    torch.cuda.synchronize()
    tms = e0.elapsed_time(e1) / 20
    tslab.close()
    sb = w["batch"] * s * w["N"] ** 3 * 4
    tbytes = 2 * (sb * (1 + 2 / 4) + sb) + 3 * sb
    return {"workload": "DG slab: 64 elements x 4 GLL nodes on [0, 1], diffuse walls u_y = -+0.3, T = 1, "
                        "the slab species/kernel/grid above, noise-free bi-Maxwellians, SSP-RK2 dt = 2e-4",
            "ms_per_step": round(ms, 3), "steps": steps + 1,
            "node_steps_per_s": round(w["batch"] / (ms * 1e-3), 1),
            "operator_evals_per_s": round(2 * w["batch"] * s * s / (ms * 1e-3), 1), "finite": ok,
            "mass_drift_between_walls": [float(abs(a / b - 1)) for a, b in zip(m1, m0)],
            "transport_only_ms_per_step": round(tms, 4),
            "transport_roofline": {"bound": "hbm", "achieved": round(tbytes / (tms * 1e-3) / 1e9, 1),
                                   "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                                   "frac": round(tbytes / (tms * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4),
                                   "bytes_per_step": tbytes}}


def dealias_leg(torch, dev, f32, w, calls):
    """The slab workload with eq. (sum) read as a linear convolution (spectra zero-padded
    to 3N/2 = 48; the padded spectra are not Hermitian, so the gain transforms them
    unpaired)."""
    from paper_1903_03056_amd import CollisionPlan
    s = len(w["masses"])
    plan = CollisionPlan(w["masses"], w["N"], w["L"], w["M"], w["n_rho"], omega=w["omega"], precision="f32",
                         dealias=True)
    f = torch.tensor(f32, device=dev)
    ws = torch.empty(plan.workspace_bytes(64), dtype=torch.uint8, device=dev)
    Q = torch.empty_like(f)
    plan.collide(f, out=Q, workspace=ws)
    torch.cuda.synchronize()
    stage = np.zeros(5)
    st = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(calls):
        _, ms = plan.collide_timed(f, out=Q, workspace=ws)
        stage += np.array(ms)
    e1.record(st)
    torch.cuda.synchronize()
    ms_call = e0.elapsed_time(e1) / calls
    stage /= calls
    NI = 3 * w["N"] // 2
    flops = w["batch"] * gain_flops_per_node_vss(NI, w["M"], w["n_rho"], s)
    return {"roofline_gain": {"bound": "alu", "achieved": round(flops / (stage[1] * 1e-3) / 1e12, 3),
                              "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                              "frac": round(flops / (stage[1] * 1e-3) / 1e12 / PEAK_FP32_VECTOR_TFLOPS, 4),
                              "flop_model": "the padded gain as one complex product per direction on 48^3"},
            "workload": "the slab workload (256 nodes, N=32, M=12, N_rho=16, FP32) with the linear (dealiased) "
                        "convolution, padded to 48^3, 64-node workspace slices",
            "value": round(w["batch"] * s * s / (ms_call * 1e-3), 1), "unit": "evals/s", "calls": calls,
            "ms_per_call": round(ms_call, 3),
            "stages_ms": {"forward_pad_interpolant": round(stage[0], 3), "gain_48": round(stage[1], 3),
                          "kept_modes_and_loss_spectrum": round(stage[2], 3),
                          "loss_product_and_inverse": round(stage[3], 3), "real_part": round(stage[4], 3)}}


def relax_leg(torch, dev, plan, f32, w, steps, dt=0.01):
    """SSP-RK2 time stepping of the slab workload (two projected operator evaluations
    per step, all on the device), timed with events around each call."""
    s = len(w["masses"])
    f = torch.tensor(f32, device=dev)
    ws = torch.empty(plan.relax_workspace_bytes(w["batch"]), dtype=torch.uint8, device=dev)
    plan.relax(f, dt, 1, workspace=ws)      # warm-up, and the state checked against the oracle
    torch.cuda.synchronize()
    got = f[0].double().cpu().numpy()
    st = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    plan.relax(f, dt, steps, workspace=ws)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    res = {"workload": "the slab above advanced by SSP-RK2 (dt = 0.01), two projected collide calls per step",
           "ms_per_step": round(ms, 3), "steps": steps,
           "operator_evals_per_s": round(2 * w["batch"] * s * s / (ms * 1e-3), 1)}
    check = dict(leg="ssprk2_relax", key="node 0 after one step", f=f32[0].astype(np.float64), got=got,
                 masses=w["masses"], omega=w["omega"], Ls=(w["L"],) * s, N=w["N"], M=w["M"], nrho=w["n_rho"],
                 dt=dt)
    return res, [check]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="leave out the plain per-point FP64 comparison leg (not part of the timed step)")
    ap.add_argument("--no-extra", action="store_true",
                    help="leave out the uneven-batch, species-grid, SSP-RK2 and measured-ceiling legs")
    ap.add_argument("--only-leg", choices=["vss_slab", "dg_slab", "dealiased_slab", "uneven_group_graph",
                                           "heavy_light_species_grids", "serving"], default=None,
                    help="run only the named extra workload and print its JSON (for profiling)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one plain device copy of 2 x 256 MiB first (calibrates HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only; the batch of independent nodes would be "
              "sharded across GPUs with no collective, which is not run here.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1903_03056_amd import CollisionPlan, tile_candidates
    from synth import inputs as I

    if args.only_leg == "vss_slab":
        log("VSS kernels only")
        print(json.dumps({"vss_slab": vss_leg(torch, torch.device("cuda:0"), args.steps)}), flush=True)
        return
    if args.only_leg == "uneven_group_graph":
        log("uneven batch only")
        print(json.dumps({args.only_leg: group_leg(torch, torch.device("cuda:0"), args.steps)[0]}), flush=True)
        return
    if args.only_leg == "serving":
        log("serving loop only")
        print(json.dumps({"serving": serving_leg(torch, torch.device("cuda:0"))}), flush=True)
        return
    if args.only_leg == "heavy_light_species_grids":
        log("heavy/light species grids only")
        print(json.dumps({args.only_leg: species_grid_leg(torch, torch.device("cuda:0"), args.steps)[0]}), flush=True)
        return
    if args.only_leg in ("dg_slab", "dealiased_slab"):
        w = WORKLOAD
        dev = torch.device("cuda:0")
        if args.only_leg == "dg_slab":
            plan = CollisionPlan(w["masses"], w["N"], w["L"], w["M"], w["n_rho"], omega=w["omega"], precision="f32")
            res = slab_leg(torch, dev, plan, w, args.steps)
        else:
            f32 = I.draw_bimaxwellian_batch(np.random.default_rng(w["seed"]), w["batch"], len(w["masses"]), w["N"],
                                            w["L"], w["masses"], noise=w["noise"]).astype(np.float32)
            res = dealias_leg(torch, dev, f32, w, args.steps)
        print(json.dumps({args.only_leg: res}), flush=True)
        return

    w = WORKLOAD
    s = len(w["masses"])
    rng = np.random.default_rng(w["seed"])
    f64 = I.draw_bimaxwellian_batch(rng, w["batch"], s, w["N"], w["L"], w["masses"], noise=w["noise"])
    f32 = f64.astype(np.float32)

    t0 = time.perf_counter()
    plan = CollisionPlan(w["masses"], w["N"], w["L"], w["M"], w["n_rho"], omega=w["omega"], precision="f32")
    precompute_s = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    f = torch.tensor(f32, device=dev)
    ws = plan.workspace(w["batch"], dev)
    Q = torch.empty_like(f)
    Qc = torch.empty(f.shape, dtype=torch.float64, device=dev)
    st = torch.cuda.current_stream(dev)

    if args.copy_probe:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {src.numel() * 4} bytes read + {dst.numel() * 4} bytes written")
        del src, dst
    log(f"slab: {args.warmup} warm-up and {args.steps} timed steps")
    for _ in range(args.warmup):
        plan.collide(f, out=Q, workspace=ws)
        plan.conserve(Q, out=Qc)
    torch.cuda.synchronize()

    stage_sum = np.zeros(5)
    cons_ms, step_ms = [], []
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        e0, e1, e2 = ev[k]
        e0.record(st)
        _, ms = plan.collide_timed(f, out=Q, workspace=ws)
        e1.record(st)
        plan.conserve(Q, out=Qc)
        e2.record(st)
        stage_sum += np.array(ms)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    for e0, e1, e2 in ev:
        step_ms.append(e0.elapsed_time(e2))
        cons_ms.append(e1.elapsed_time(e2))
    ms_per_step = (t_end - t_start) * 1e3 / args.steps
    evals = w["batch"] * s * s
    value = evals / (ms_per_step / 1e3)

    stage_avg = stage_sum / args.steps
    gain_ms = stage_avg[1]
    flop_node = gain_flops_per_node(w["N"], w["M"], w["n_rho"], s)
    achieved = flop_node * w["batch"] / (gain_ms / 1e3) / 1e12
    geometry = tuple(plan.tile) if plan.tile else tuple(tile_candidates(w["N"], "f32")[0])
    traffic = load_traffic()
    cons_avg = float(np.mean(cons_ms))
    cons_bytes = w["batch"] * s * w["N"] ** 3 * (4 + 8)
    cons_gbps = cons_bytes / (cons_avg / 1e3) / 1e9

    out = {
        "metric": "collision evals/s (node x ordered species pair) at N=32, M=12",
        "value": round(value, 2),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1D DG slab, 64 elements x 4 nodes = 256 points, 2 species m=(1,2), VHS omega=0.74, "
                               "N=32, L=6, M=12, N_rho=16, bi-Maxwellian + 1e-2 noise, seed 2; FP32 collide + "
                               "FP64 conservation projection",
                   "batch": w["batch"], "species": s, "N": w["N"], "M": w["M"], "n_rho": w["n_rho"]},
        "latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 4),
                       "p99": round(float(np.percentile(step_ms, 99)), 4)},
        "stages_ms": {"forward_fft": round(stage_avg[0], 4), "gain": round(stage_avg[1], 4),
                      "radial_loss": round(stage_avg[2], 4), "inverse_xy": round(stage_avg[3], 4),
                      "inverse_z_combine": round(stage_avg[4], 4), "conserve_fp64": round(cons_avg, 4)},
        "roofline": {"bound": "mfma" if geometry[1] == 0 else "alu",
                     "kernel": "mfma::gain_kernel" if geometry[1] == 0 else "gain_kernel",
                     "geometry": list(geometry), "achieved": round(achieved, 3),
                     "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
                     "traffic": traffic, "flop_per_launch": flop_node * w["batch"],
                     "flop_model": "the FP32 work of the spectral gain (FFT model), against the FP32 "
                                   "peak (vector = matrix, 157.3 TFLOP/s)"},
        "conserve_roofline": {"bound": "hbm", "achieved": round(cons_gbps, 1), "peak": PEAK_HBM_GBPS,
                              "unit": "GB/s", "frac": round(cons_gbps / PEAK_HBM_GBPS, 4),
                              "bytes_per_launch": cons_bytes},
        "precompute_s": round(precompute_s, 3),
        "rel_linf_vs_stored_oracle_samples": stored_oracle_errors("slab_N32", Q),
    }
    if geometry[1] == 0:
        mf = mfma_flops_per_launch(w["batch"], w["N"], w["M"], w["n_rho"], s)
        out["roofline"]["matrix_cores"] = {
            "executed_flop_per_launch": mf, "achieved": round(mf / (gain_ms / 1e3) / 1e12, 1),
            "peak": PEAK_FP16_MFMA_TFLOPS, "unit": "TFLOP/s (FP16 dense, the split products)",
            "frac": round(mf / (gain_ms / 1e3) / 1e12 / PEAK_FP16_MFMA_TFLOPS, 4)}
    Qh = Q.double().cpu().numpy()
    Qch = Qc[:4].cpu().numpy()
    # the plain per-point FP64 GPU path on the first nodes of the same workload
    plain_nodes = 0 if args.no_plain else 2
    if plain_nodes:
        log("plain FP64 path")
        plan64 = CollisionPlan(w["masses"], w["N"], w["L"], w["M"], w["n_rho"], omega=w["omega"], precision="f64")
        f64d = torch.tensor(f32[:plain_nodes].astype(np.float64), device=dev)
        Qp = plan64.collide_plain(f64d[:1])          # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Qp = plan64.collide_plain(f64d)
        torch.cuda.synchronize()
        plain_s = time.perf_counter() - t0
        out["plain_fp64_path"] = {"value": round(plain_nodes * s * s / plain_s, 2), "unit": "evals/s",
                                  "sample": f"first {plain_nodes} nodes, one node per pass, unfused FP64 kernels"}
    if not args.no_extra:
        log("measured ceilings")
        peaks = measured_peaks(torch, dev)
        out["measured_peaks"] = peaks
        out["roofline"]["frac_of_measured_fma"] = round(achieved / peaks["valu_fp32_fma_TFLOPs"], 4)
        log("uneven batch in one graph")
        extra, checks = {}, []
        extra["uneven_group_graph"], c = group_leg(torch, dev, 20)
        checks += c
        log("species-specific grids")
        extra["heavy_light_species_grids"], c = species_grid_leg(torch, dev, 3)
        checks += c
        log("VSS kernels")
        extra["vss_slab"] = vss_leg(torch, dev, 5)
        log("dealiased form")
        extra["dealiased_slab"] = dealias_leg(torch, dev, f32, w, 2)
        log("DG slab")
        extra["dg_slab"] = slab_leg(torch, dev, plan, w, 10)
        log("SSP-RK2 stepping")
        extra["ssprk2_relax"], c = relax_leg(torch, dev, plan, f32, w, 10)
        checks += c
        log("serving loop")
        extra["serving"] = serving_leg(torch, dev)
        out["workloads"] = extra
    else:
        checks = []

    def rel_err(a, ref):
        num = np.abs(a - ref).reshape(s, -1).max(1)
        return float(np.max(num / np.abs(ref).reshape(s, -1).max(1)))

    if not args.no_cpu_baseline:
        log("oracle on the host cores")
        from oracle import moments as OM
        base, outs = cpu_baseline(f32.astype(np.float64))
        out["cpu_baseline"] = base
        out["max_rel_linf_vs_oracle"] = max(rel_err(Qh[b], ref) for b, ref in enumerate(outs))
        out["conservation_residual_after_fp64_projection"] = float(max(
            OM.conservation_residual(Qch[b], w["masses"], (w["L"],) * s).max() for b in range(Qch.shape[0])))
        if plain_nodes:
            Qph = Qp.cpu().numpy()
            out["plain_fp64_path"]["max_rel_linf_vs_oracle"] = max(
                rel_err(Qph[b], outs[b]) for b in range(min(plain_nodes, len(outs))))
        # sampled nodes of the other workloads against the oracle
        from oracle import grids as OG, spectral as OS, stepping as OT
        for c in checks:
            prob = OS.vhs_problem(c["masses"], c["omega"], c["Ls"][0], c["N"], c["M"], c["nrho"])
            if "dt" in c:
                ref = OT.ssprk2(c["f"], OT.collision_rhs(prob), c["dt"], 1)
            elif len(set(c["Ls"])) > 1:
                ref = OG.collide(c["f"], prob, c["Ls"])
            else:
                ref = OS.collide(c["f"], prob)
            ns = len(c["masses"])
            err = float(np.max(np.abs(c["got"] - ref).reshape(ns, -1).max(1) / np.abs(ref).reshape(ns, -1).max(1)))
            out["workloads"][c["leg"]].setdefault("max_rel_linf_vs_oracle", {})[c["key"]] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
