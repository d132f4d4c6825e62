"""Benchmark of the batched multi-species collision operator on one MI355X.

Workload (one "step"): the 1-D DG slab of 64 elements x 4 GLL nodes = 256 independent
spatial points, 2 species with masses (1, 2), VHS omega = 0.74, N = 32, L = 6, M = 12
(icosahedron), N_rho = 16, seeded bi-Maxwellians with 1e-2 uniform noise.  A step is
the whole hot path: forward transforms, gain (rho, sigma) loop, radial sum and loss,
inverse transforms and combination (dgfs_collide), then the FP64 conservation
projection (dgfs_conserve).  Inputs are resident in device memory before timing.

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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="leave out the plain per-point FP64 comparison leg (not part of the timed step)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one plain device copy of 2 x 256 MiB first (calibrates HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only; the batch of independent nodes would be "
              "sharded across GPUs with no collective, which is not run here.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1903_03056_amd import CollisionPlan
    from synth import inputs as I

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
                      "radial_loss": round(stage_avg[2], 4), "inverse_fft": round(stage_avg[3], 4),
                      "combine": round(stage_avg[4], 4), "conserve_fp64": round(cons_avg, 4)},
        "roofline": {"bound": "alu", "kernel": "gain_kernel", "achieved": round(achieved, 3),
                     "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
                     "traffic": traffic, "flop_per_launch": flop_node * w["batch"]},
        "conserve_roofline": {"bound": "hbm", "achieved": round(cons_gbps, 1), "peak": PEAK_HBM_GBPS,
                              "unit": "GB/s", "frac": round(cons_gbps / PEAK_HBM_GBPS, 4),
                              "bytes_per_launch": cons_bytes},
        "precompute_s": round(precompute_s, 3),
    }
    # the plain per-point FP64 GPU path on the first nodes of the same workload
    plain_nodes = 0 if args.no_plain else 2
    if plain_nodes:
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

    def rel_err(a, ref):
        num = np.abs(a - ref).reshape(s, -1).max(1)
        return float(np.max(num / np.abs(ref).reshape(s, -1).max(1)))

    if not args.no_cpu_baseline:
        base, outs = cpu_baseline(f32.astype(np.float64))
        out["cpu_baseline"] = base
        Qh = Q.double().cpu().numpy()
        out["max_rel_linf_vs_oracle"] = max(rel_err(Qh[b], ref) for b, ref in enumerate(outs))
        if plain_nodes:
            Qph = Qp.cpu().numpy()
            out["plain_fp64_path"]["max_rel_linf_vs_oracle"] = max(
                rel_err(Qph[b], outs[b]) for b in range(min(plain_nodes, len(outs))))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
