"""GPU parity at the full sizes the benchmark times, in the launch configuration it uses,
against FP64 oracle results sampled on nodes spread over each batch (see
tests/golden/make_oracle_samples.py: the oracle is minutes per node at these sizes, so
its values are stored, per node the largest-|Q| points, each pair's largest point and a
seeded uniform sample of about 450 grid points per species, with the exact max |Q| and
loss scale over the whole grid).

Measures, as in the other parity tests:
* summed result Q^i: max |Q - Q_ref| / max_v |Q_ref| per (node, species), <= 1e-5 (FP32);
* pair-resolved Q^{ij}: max |Q^{ij} - Q^{ij}_ref| over the pair's loss scale
  max_v |f^i nu^{ij}| (a like pair of near-equilibrium data is a small difference of gain
  and loss, so its own maximum is no scale for FP32 rounding), <= 1e-5.
For the heavy/light workload (Maxwellians at rest, near equilibrium: Q^i is a few per cent
of its gain and loss terms) the summed result is measured against the loss scale too,
max_j max_v |f^i nu^{ij}| (a lower bound of max_v |f^i sum_j nu^{ij}|, nu^{ij} >= 0), and
its error relative to max_v |Q^i| is printed beside it.  The distributions are printed."""
import math

import numpy as np
import pytest

from synth import inputs as I

import _golden as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _pairs_of(plan, ft, nodes, **kw):
    """Pair-resolved results of the sampled nodes, {node: host array [s][s][N^3]}: the
    nodes collided as one batch (a node's result does not depend on its batch)."""
    sel = torch.tensor(np.asarray(nodes), device="cuda")
    Qp = plan.collide(ft[sel].contiguous(), pairs=True, **kw).double().cpu().numpy()
    return {int(b): Qp[k] for k, b in enumerate(nodes)}


def _check_nodes(name, f32, Q, Qp, tol=1e-5, summed_scale="qmax"):
    """Compare the sampled nodes of workload `name`; f32, Q: host arrays of the whole
    batch (inputs, summed result), Qp: {node: pair-resolved result} or None.
    summed_scale: "qmax" (max_v |Q^i_ref|) or "loss" (max_j of the pairs' loss scales)."""
    d, meta = G.load(name)
    nodes = d["nodes"]
    summed, pairs, vs_qmax = [], [], []
    for k, b in enumerate(nodes):
        G.check_inputs(f32[b], d["fsum"][k])
        es = G.summed_errors(Q[b], d["idx"][k], d["qp"][k], d["qmax"][k])
        if summed_scale == "loss":
            vs_qmax.append(es)
            es = es * d["qmax"][k] / d["loss"][k].max(axis=1)
        summed.append(es)
        if Qp is not None:
            pairs.append(G.pair_errors(Qp[int(b)], d["idx"][k], d["qp"][k], d["loss"][k]))
        print(f"{name} node {int(b)} (XCD {int(b) % 8}): summed {np.array2string(es, precision=3)}"
              + (f" pairs/loss {np.array2string(pairs[-1].ravel(), precision=3)}" if Qp is not None else ""),
              flush=True)
    print(G.describe(f"{name} summed" + (" over the loss scale" if summed_scale == "loss" else ""), summed),
          flush=True)
    if vs_qmax:
        print(G.describe(f"{name} summed over max |Q| (reported, not asserted)", vs_qmax), flush=True)
        print(f"{name} max |Q^i| / loss scale: "
              f"{np.array2string(d['qmax'] / d['loss'].max(axis=2), precision=3)}", flush=True)
    if Qp is not None:
        print(G.describe(f"{name} pairs over the loss scale", pairs), flush=True)
    assert np.max(summed) <= tol
    if Qp is not None:
        assert np.max(pairs) <= tol
    return nodes


def test_slab_N32_full_batch_vs_oracle_samples():
    """The 256-node N = 32 slab (M = 12, N_rho = 16, omega = 0.74, bi-Maxwellian + 1e-2
    noise, FP32) in one pass with the default tile: 16 nodes covering every residue mod 8."""
    _require_gpu()
    from paper_1903_03056_amd import CollisionPlan
    print("[case] full size: slab N=32 B=256", flush=True)
    c = I.config(2)
    f = I.draw_bimaxwellian_batch(np.random.default_rng(c["seed"]), c["batch"], c["s"], c["N"], c["L"],
                                  c["masses"], noise=c["noise"]).astype(np.float32)
    plan = CollisionPlan(c["masses"], c["N"], c["L"], c["M"], c["nrho"], omega=c["omega"], precision="f32")
    ft = torch.tensor(f, device="cuda")
    ws = plan.workspace(c["batch"])
    Q = plan.collide(ft, workspace=ws).cpu().numpy()
    Qp = _pairs_of(plan, ft, G.load("slab_N32")[0]["nodes"])
    nodes = _check_nodes("slab_N32", f, Q, Qp)
    assert set(int(b) % 8 for b in nodes) == set(range(8))


def test_heavy_light_full_batch_vs_oracle_samples():
    """1024 nodes, m = (1, 32.75) on species grids L = (6, 1.0484), hard spheres, N = 48,
    M = 24, N_rho = 24, FP32, autotuned tile, 256-node workspace slices: 16 nodes spread
    over the batch (the last in the final slice), summed and pair-resolved."""
    _require_gpu()
    from paper_1903_03056_amd import CollisionPlan
    print("[case] full size: heavy/light species grids N=48 B=1024", flush=True)
    c = I.config(3)
    Ls = tuple(c["L"] * math.sqrt(1.0 / m) for m in c["masses"])
    f = I.draw_config3_batch(np.random.default_rng(c["seed"]), c["batch"], c["N"], Ls, c["masses"]).astype(np.float32)
    plan = CollisionPlan(c["masses"], c["N"], Ls, c["M"], c["nrho"], omega=c["omega"], precision="f32", tile="auto")
    print(f"tile {plan.tile}", flush=True)
    ft = torch.tensor(f, device="cuda")
    ws = torch.empty(plan.workspace_bytes(256), dtype=torch.uint8, device="cuda")
    Q = plan.collide(ft, workspace=ws).cpu().numpy()
    Qp = _pairs_of(plan, ft, G.load("heavy_light_N48")[0]["nodes"], workspace=ws)
    _check_nodes("heavy_light_N48", f, Q, Qp, summed_scale="loss")


def test_uneven_group_graph_vs_oracle_samples():
    """512 nodes at N = 24, 256 at N = 32 and 64 at N = 48, three species (1, 2, 4),
    M = 12, N_rho = N/2, autotuned tiles, captured in one hipGraph and replayed: 8 nodes
    of the N = 24 and N = 32 classes and 4 of the N = 48 class against the oracle, and
    every class equal bit for bit to its plan alone."""
    _require_gpu()
    from paper_1903_03056_amd import CollisionGroup, CollisionPlan
    print("[case] full size: uneven group graph 512@24 + 256@32 + 64@48", flush=True)
    c = I.config(4)
    fs = [x.astype(np.float32) for x in I.draw_uneven_groups(c["seed"], c["groups"], c["s"], c["L"], c["masses"])]
    plans = [CollisionPlan(c["masses"], N, c["L"], c["M"], N // 2, omega=c["omega"], precision="f32", tile="auto")
             for N, _ in c["groups"]]
    print(f"tiles {[p.tile for p in plans]}", flush=True)
    group = CollisionGroup(plans)
    ft = [torch.tensor(x, device="cuda") for x in fs]
    graph, outs = group.capture(ft)
    graph.launch()
    graph.launch()
    graph.stream.synchronize()
    for (N, B), plan, x, q, fh in zip(c["groups"], plans, ft, outs, fs):
        alone = plan.collide(x)
        torch.cuda.synchronize()
        assert torch.equal(alone, q), N
        _check_nodes(f"uneven_N{N}", fh, q.cpu().numpy(), None)
    graph.close()
    group.close()


def test_vss_slab_full_batch_vs_oracle_samples():
    """The slab shape with the argon-krypton VSS kernels (omega 0.81/0.805/0.8, alpha
    1.4/1.36/1.32, m2/m1 = 139.1/66.3), 256 nodes, N = 32, M = 12, N_rho = 16, FP32: 8
    nodes against the oracle, summed and pair-resolved."""
    _require_gpu()
    from paper_1903_03056_amd import CollisionPlan, vss_kernel
    print("[case] full size: VSS slab N=32 B=256", flush=True)
    d, meta = G.load("vss_slab_N32")
    masses = tuple(meta["masses"])
    omega = ((0.81, 0.805), (0.805, 0.8))
    alpha = ((1.4, 1.36), (1.36, 1.32))
    f = I.draw_bimaxwellian_batch(np.random.default_rng(meta["seed"]), meta["batch"], 2, meta["N"], meta["L"], masses,
                                  noise=meta["noise"]).astype(np.float32)
    plan = CollisionPlan(masses, meta["N"], meta["L"], meta["M"], meta["nrho"], kernel=vss_kernel(masses, omega, alpha),
                         precision="f32")
    ft = torch.tensor(f, device="cuda")
    Q = plan.collide(ft, workspace=plan.workspace(meta["batch"])).cpu().numpy()
    Qp = _pairs_of(plan, ft, d["nodes"])
    _check_nodes("vss_slab_N32", f, Q, Qp)
