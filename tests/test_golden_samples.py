"""The stored oracle samples (tests/golden/oracle_*.npz, written by
tests/golden/make_oracle_samples.py from the oracle alone) are what the oracle gives:
one node of the N = 32 slab is evaluated again here and must agree with the stored
values to round-off, and every file holds the fields the GPU tests read, with sample
indices inside the grid and the exact maxima at least as large as any sampled value."""
import os

import numpy as np
import pytest

from oracle import spectral as OS
from synth import inputs as I

import _golden as G

NAMES = ["slab_N32", "heavy_light_N48", "vss_slab_N32", "uneven_N24", "uneven_N32", "uneven_N48"]


@pytest.mark.parametrize("name", NAMES)
def test_sample_files_are_consistent(name):
    d, meta = G.load(name)
    n, s, K = d["idx"].shape
    assert d["qp"].shape == (n, s, s, K) and d["qmax"].shape == (n, s) and d["loss"].shape == (n, s, s)
    assert len(d["nodes"]) == n == len(meta["nodes"])
    assert d["idx"].min() >= 0 and d["idx"].max() < meta["N"] ** 3
    for k in range(n):
        summed = d["qp"][k].sum(axis=1)
        assert np.all(np.abs(summed).max(axis=1) <= d["qmax"][k] * (1 + 1e-12))
        assert np.all(np.abs(d["qp"][k]).max(axis=2) <= d["qpmax"][k] * (1 + 1e-12))
        # the largest |Q^i| point is among the samples
        assert np.allclose(np.abs(summed).max(axis=1), d["qmax"][k], rtol=1e-12)


def test_serve_file_is_consistent():
    d, meta = G.load("serve_traj")
    for k, req in enumerate(meta["requests"]):
        s = len(req["masses"])
        assert d[f"r{k}_idx"].shape[0] == s and d[f"r{k}_qp"].shape[:2] == (s, 1)
        assert np.allclose(np.abs(d[f"r{k}_qp"][:, 0]).max(axis=1), d[f"r{k}_qmax"], rtol=1e-12)


@pytest.mark.slow
def test_one_slab_node_recomputed_by_the_oracle():
    """Node 17 of the slab workload (N = 32, M = 12, N_rho = 16): the oracle's result now
    equals the stored samples (FFT thread counts may change the rounding order)."""
    d, meta = G.load("slab_N32")
    k = int(np.flatnonzero(d["nodes"] == 17)[0])
    f = I.draw_bimaxwellian_batch(np.random.default_rng(meta["seed"]), meta["batch"], 2, meta["N"], meta["L"],
                                  tuple(meta["masses"]), noise=meta["noise"])[17].astype(np.float32).astype(np.float64)
    G.check_inputs(f, d["fsum"][k])
    prob = OS.vhs_problem(tuple(meta["masses"]), meta["omega"], meta["L"], meta["N"], meta["M"], meta["nrho"])
    Qp = OS.collide_pairs(f, prob).reshape(2, 2, -1)
    idx = d["idx"][k]
    for i in range(2):
        for j in range(2):
            np.testing.assert_allclose(Qp[i, j, idx[i]], d["qp"][k][i, j], rtol=0, atol=1e-13 * d["qmax"][k][i])
    assert np.allclose(np.abs(Qp.sum(axis=1)).max(axis=1), d["qmax"][k], rtol=1e-12)
