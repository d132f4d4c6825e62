"""Reading the sampled oracle results of tests/golden/oracle_<name>.npz (written by
tests/golden/make_oracle_samples.py, which calls only the oracle) and comparing device
results with them."""
from __future__ import annotations

import json
import os

import numpy as np

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name: str):
    """(arrays, meta) of one workload's samples."""
    d = np.load(os.path.join(HERE, f"oracle_{name}.npz"), allow_pickle=False)
    return d, json.loads(str(d["meta"]))


def check_inputs(f_node, fsum):
    """The test's FP32-rounded input of one node is the one the samples were taken on
    (the sums of every species field agree to round-off)."""
    got = np.asarray(f_node, dtype=np.float64).reshape(len(fsum), -1).sum(axis=1)
    np.testing.assert_allclose(got, fsum, rtol=1e-12, atol=0.0)


def summed_errors(Q_node, idx, qp, qmax):
    """Per species max over the samples of |Q - Q_ref| / max_v |Q_ref| (Q_ref summed over j)."""
    s = len(qmax)
    q = np.asarray(Q_node, dtype=np.float64).reshape(s, -1)
    ref = qp.sum(axis=1)                      # [s][K]
    err = np.array([np.abs(q[i, idx[i]] - ref[i]).max() for i in range(s)])
    return err / qmax


def pair_errors(Qp_node, idx, qp, scale):
    """Per ordered pair max over the samples of |Q^{ij} - Q^{ij}_ref| / scale[i][j]."""
    s = qp.shape[0]
    q = np.asarray(Qp_node, dtype=np.float64).reshape(s, s, -1)
    err = np.array([[np.abs(q[i, j, idx[i]] - qp[i, j]).max() for j in range(s)] for i in range(s)])
    return err / scale


def describe(label, errs):
    """One line with the distribution of the errors (printed next to the assertion)."""
    e = np.asarray(errs, dtype=np.float64).ravel()
    return (f"{label}: n={e.size} max {e.max():.3e} p50 {np.percentile(e, 50):.3e} "
            f"p90 {np.percentile(e, 90):.3e} min {e.min():.3e}")
