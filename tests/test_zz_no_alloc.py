"""dgfs_collide_static: the collide of dgfs_collide with the library's own static device
workspace (for callers that cannot allocate), through the C ABI.  Its results equal
dgfs_collide's bit for bit (nodes are independent, so the slicing a workspace size
implies does not change any value) on two calls in a row, the second with a smaller
input; a plan whose single node needs more than the static workspace is refused."""
import ctypes

import numpy as np
import pytest

from synth import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _static(plan, f):
    """dgfs_collide_static called through the C ABI (ctypes, no binding method)."""
    from paper_1903_03056_amd import _lib
    lib = _lib.load()
    fn = lib.dgfs_collide_static
    fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    fn.restype = ctypes.c_int32
    Q = torch.empty_like(f)
    st = torch.cuda.current_stream(f.device)
    _lib.check(fn(plan._plan, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(Q.data_ptr()), f.shape[0],
                  ctypes.c_void_p(st.cuda_stream)), "dgfs_collide_static")
    return Q


CASES = {
    # 40 nodes of the N = 32 slab shape: more than the static workspace holds in one pass
    "slab N=32 fp32": dict(masses=(1.0, 2.0), N=32, L=6.0, M=12, nrho=16, kw=dict(omega=0.74, precision="f32"),
                           batch=40, noise=1e-2),
    "species grids N=24 fp32": dict(masses=(1.0, 32.75), N=24, L=(6.0, 6.0 * np.sqrt(1.0 / 32.75)), M=24, nrho=12,
                                    kw=dict(omega=0.5, precision="f32"), batch=9, noise=0.0),
    "VSS N=16 fp64": dict(masses=(1.0, 2.0), N=16, L=6.0, M=12, nrho=8, kw=dict(precision="f64"), batch=5,
                          noise=1e-2, vss=True),
}


@pytest.mark.parametrize("name", list(CASES))
def test_collide_static_equals_collide(name):
    _require_gpu()
    from paper_1903_03056_amd import CollisionPlan, vss_kernel
    c = CASES[name]
    print(f"[case] collide_static {name}", flush=True)
    kw = dict(c["kw"])
    if c.get("vss"):
        kw["kernel"] = vss_kernel(c["masses"], 0.8, 1.4)
    plan = CollisionPlan(c["masses"], c["N"], c["L"], c["M"], c["nrho"], **kw)
    rng = np.random.default_rng(len(name))
    f = I.draw_bimaxwellian_batch(rng, c["batch"], len(c["masses"]), c["N"], c["L"], c["masses"], noise=c["noise"])
    ft = torch.tensor(f, dtype=plan.dtype, device="cuda")
    for f_in in (ft, (1.5 * ft[1:4]).contiguous()):     # second call: a smaller input
        ref = plan.collide(f_in)
        got = _static(plan, f_in)
        via_binding = plan.collide_static(f_in)
        torch.cuda.synchronize()
        assert torch.equal(ref, got), f_in.shape[0]
        assert torch.equal(ref, via_binding), f_in.shape[0]


def test_collide_static_refuses_oversized_plan():
    """FP64, N = 48, s = 3, M = 24 (nine classes), N_rho = 32: one node needs about 276 MB
    of workspace, more than the 256 MiB static array."""
    _require_gpu()
    from paper_1903_03056_amd import CollisionPlan
    from paper_1903_03056_amd._lib import DGFS_ENOMEM, DgfsError
    print("[case] collide_static oversized plan", flush=True)
    from paper_1903_03056_amd import _lib
    plan = CollisionPlan((1.0, 2.0, 4.0), 48, 6.0, 24, 32, omega=0.74, precision="f64")
    assert _lib.load().dgfs_static_workspace_bytes() == 256 << 20
    assert plan.workspace_bytes(1) > 256 << 20
    f = torch.zeros((1, 3, 48, 48, 48), dtype=torch.float64, device="cuda")
    with pytest.raises(DgfsError) as e:
        _static(plan, f)
    assert e.value.status == DGFS_ENOMEM
