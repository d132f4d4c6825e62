"""Autotuner for the gain-kernel geometry (tile) of a collision problem.

The gain kernel is compiled for a few geometries per (N, precision): the number CH of
x-chunks a field is split into (an N/CH-point x-FFT after a CH-way decimation in
frequency) and the number CZ of thread groups sharing a y/z pencil (N/CZ-point FFTs
after a CZ-way split).  They trade FFT work, LDS capacity and occupancy differently on
each grid, so the tuner times every compiled candidate on the current device with a
synthetic batch of the problem's shape and keeps the fastest.  Results are cached in
JSON (DGFS_TUNE_CACHE, default ~/.cache/dgfs/tiles.json) keyed by device architecture,
N, precision, M, N_rho and the species count.
"""
from __future__ import annotations

import json
import os

import numpy as np


def cache_path() -> str:
    return os.environ.get("DGFS_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "dgfs",
                                                             "tiles.json")


def _load():
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(cache):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _key(N, precision, M, n_rho, s):
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    return f"{arch}|N={N}|{precision}|M={M}|nrho={n_rho}|s={s}"


def tune(masses, N, L, M, n_rho, kernel, precision="f32", batch=32, reps=3, seed=0):
    """Time every compiled geometry; returns {(ch, cz): median gain-kernel ms}."""
    import torch

    from synth import inputs as I

    from .collision import CollisionPlan, tile_candidates

    s = len(masses)
    rng = np.random.default_rng(seed)
    f = I.draw_bimaxwellian_batch(rng, batch, s, N, L, masses)
    dt = torch.float64 if precision in ("f64", "fp64", "float64") else torch.float32
    ft = torch.tensor(f, dtype=dt, device="cuda")
    times = {}
    for tile in tile_candidates(N, precision):
        plan = CollisionPlan(masses, N, L, M, n_rho, kernel=kernel, precision=precision, tile=tile)
        out = torch.empty_like(ft)
        ws = plan.workspace(batch)
        plan.collide(ft, out=out, workspace=ws)
        samples = [plan.collide_timed(ft, out=out, workspace=ws)[1][1] for _ in range(reps)]
        times[tuple(tile)] = float(np.median(samples))
        plan.close()
    return times


def best_tile(masses, N, L, M, n_rho, kernel, precision="f32", batch=32, reps=3):
    """The fastest geometry for this problem shape (cached)."""
    cache = _load()
    key = _key(N, precision, M, n_rho, len(masses))
    if key in cache:
        return tuple(cache[key]["tile"])
    times = tune(masses, N, L, M, n_rho, kernel, precision, batch, reps)
    best = min(times, key=times.get)
    cache[key] = {"tile": list(best), "gain_ms": {f"{k[0]}x{k[1]}": v for k, v in times.items()},
                  "batch": batch}
    _store(cache)
    return best
