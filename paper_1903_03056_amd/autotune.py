"""Autotuner for the gain-kernel geometry (tile) of a collision problem.

The gain kernel is compiled for a few geometries per (N, precision): the number CH of
x-chunks a field is split into (an N/CH-point x-FFT after a CH-way decimation in
frequency) and the number CZ of thread groups sharing a y/z pencil (N/CZ-point FFTs
after a CZ-way split).  They trade FFT work, LDS capacity and occupancy differently on
each grid, so the tuner times every compiled candidate on the current device with a
synthetic batch of the problem's shape and keeps the fastest.  Results are cached in
JSON (DGFS_TUNE_CACHE, default ~/.cache/dgfs/tiles.json) keyed by device architecture,
a digest of the built library, N, precision, M, N_rho, the species count, the kernel
family (VHS or VSS) and the species' grid layout; a cached geometry the current build no
longer compiles is tuned again.
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


_LIB_DIGEST = None


def _lib_digest() -> str:
    """SHA-256 (first 16 hex digits) of the loaded library file: a rebuild may change the
    kernels' relative speed, so tuning results are kept per build."""
    global _LIB_DIGEST
    if _LIB_DIGEST is None:
        import hashlib

        from . import _lib
        h = hashlib.sha256()
        with open(_lib.LIB_PATH, "rb") as fh:
            for block in iter(lambda: fh.read(1 << 20), b""):
                h.update(block)
        _LIB_DIGEST = h.hexdigest()[:16]
    return _LIB_DIGEST


def _key(N, precision, M, n_rho, kernel, Ls):
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    s = len(Ls)
    family = "vss" if any(kernel[i][j][1] != 1.0 for i in range(s) for j in range(s)) else "vhs"
    top = max(Ls)
    grids = ",".join(f"{x / top:.6f}" for x in Ls)
    return f"{arch}|lib={_lib_digest()}|N={N}|{precision}|M={M}|nrho={n_rho}|s={s}|{family}|grids={grids}"


def tune(masses, N, L, M, n_rho, kernel, precision="f32", batch=32, reps=3, seed=0):
    """Time every compiled geometry; returns {(ch, cz): median gain-kernel ms}.  L is one
    half-width or one per species (species-specific grids)."""
    import torch

    from synth import inputs as I

    from ._lib import DGFS_OK
    from .collision import CollisionPlan, check_problem, tile_candidates

    s = len(masses)
    Ls = tuple(float(x) for x in np.broadcast_to(np.asarray(L, dtype=np.float64), (s,)))
    rng = np.random.default_rng(seed)
    f = I.draw_bimaxwellian_batch(rng, batch, s, N, Ls, masses)
    dt = torch.float64 if precision in ("f64", "fp64", "float64") else torch.float32
    ft = torch.tensor(f, dtype=dt, device="cuda")
    times = {}
    for tile in tile_candidates(N, precision):
        # geometries the problem does not admit (the matrix-core one needs VHS kernels)
        Lsp = Ls if len(set(Ls)) > 1 else None
        if check_problem(masses, max(Ls), N, M, n_rho, kernel, precision, Lsp, tile=tile) != DGFS_OK:
            continue
        plan = CollisionPlan(masses, N, Ls, M, n_rho, kernel=kernel, precision=precision, tile=tile)
        out = torch.empty_like(ft)
        ws = plan.workspace(batch)
        plan.collide(ft, out=out, workspace=ws)
        samples = [plan.collide_timed(ft, out=out, workspace=ws)[1][1] for _ in range(reps)]
        times[tuple(tile)] = float(np.median(samples))
        plan.close()
    return times


def best_tile(masses, N, L, M, n_rho, kernel, precision="f32", batch=32, reps=3):
    """The fastest geometry for this problem shape (cached).  L: one half-width or one
    per species."""
    from .collision import tile_candidates

    s = len(masses)
    Ls = tuple(float(x) for x in np.broadcast_to(np.asarray(L, dtype=np.float64), (s,)))
    cache = _load()
    key = _key(N, precision, M, n_rho, kernel, Ls)
    compiled = [tuple(t) for t in tile_candidates(N, precision)]
    if key in cache and tuple(cache[key]["tile"]) in compiled:
        return tuple(cache[key]["tile"])
    times = tune(masses, N, Ls, M, n_rho, kernel, precision, batch, reps)
    best = min(times, key=times.get)
    cache[key] = {"tile": list(best), "gain_ms": {f"{k[0]}x{k[1]}": v for k, v in times.items()},
                  "batch": batch}
    _store(cache)
    return best
