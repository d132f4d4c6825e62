"""Python face of the collision library: plan creation and the collide / conserve calls.

PyTorch supplies device memory and streams; the arithmetic runs in libdgfs.so.
"""
from __future__ import annotations

import ctypes
from ctypes import POINTER, c_double, c_size_t, c_void_p

import numpy as np

from . import _lib
from ._lib import DGFS_FP32, DGFS_FP64, PairKernel, Problem, check, load


def pair_prefactor(mi: float, mj: float, omega: float, alpha: float = 1.0, kn0: float = 1.0) -> float:
    """C_ij of the dimensionless kernel, computed by the library (dgfs_pair_prefactor)."""
    C = c_double()
    check(load().dgfs_pair_prefactor(float(mi), float(mj), float(omega), float(alpha), float(kn0), ctypes.byref(C)),
          "dgfs_pair_prefactor")
    return C.value


def _precision_code(precision) -> int:
    if precision in ("f32", "fp32", "float32", DGFS_FP32):
        return DGFS_FP32
    if precision in ("f64", "fp64", "float64", DGFS_FP64):
        return DGFS_FP64
    raise ValueError(f"unknown precision {precision!r}")


class _ProblemHolder:
    """Keeps the ctypes arrays alive as long as the Problem struct refers to them."""

    def __init__(self, masses, L, N, M, n_rho, kernel, precision, L_species=None, tile=None, dealias=False):
        s = len(masses)
        self.mass = (c_double * s)(*masses)
        self.kern = (PairKernel * (s * s))()
        for i in range(s):
            for j in range(s):
                om, al, C = kernel[i][j]
                self.kern[i * s + j] = PairKernel(om, al, C)
        self.Ls = (c_double * s)(*L_species) if L_species is not None else None
        self.problem = Problem(s=s, mass=self.mass, L=float(L),
                               L_species=self.Ls if self.Ls is not None else None,
                               N=N, M=M, n_rho=n_rho, kernel=self.kern, precision=_precision_code(precision),
                               tile_ch=int(tile[0]) if tile else 0, tile_cz=int(tile[1]) if tile else 0,
                               dealias=1 if dealias else 0)


def vhs_kernel(masses, omega, alpha: float = 1.0, kn0: float = 1.0):
    s = len(masses)
    return [[(omega, alpha, pair_prefactor(masses[i], masses[j], omega, alpha, kn0)) for j in range(s)]
            for i in range(s)]


def vss_kernel(masses, omega, alpha, kn0: float = 1.0):
    """Kernel of eq. NVSS per ordered pair: omega and alpha are scalars or symmetric
    [s][s] tables (e.g. a mixture's like and unlike parameters)."""
    s = len(masses)
    om = np.broadcast_to(np.asarray(omega, dtype=np.float64), (s, s))
    al = np.broadcast_to(np.asarray(alpha, dtype=np.float64), (s, s))
    return [[(float(om[i, j]), float(al[i, j]), pair_prefactor(masses[i], masses[j], om[i, j], al[i, j], kn0))
             for j in range(s)] for i in range(s)]


def check_problem(masses, L, N, M, n_rho, kernel, precision="f32", L_species=None, tile=None,
                  dealias=False) -> int:
    """Host-side validation; returns the dgfs status code (0 = ok)."""
    h = _ProblemHolder(masses, L, N, M, n_rho, kernel, precision, L_species, tile=tile, dealias=dealias)
    return load().dgfs_check_problem(ctypes.byref(h.problem))


def tile_candidates(N: int, precision="f32"):
    """Gain-kernel geometries (ch, cz) compiled for (N, precision); the first is the default."""
    lib = load()
    buf = (ctypes.c_int32 * 32)()
    n = ctypes.c_int32()
    check(lib.dgfs_tile_candidates(N, _precision_code(precision), buf, 16, ctypes.byref(n)), "dgfs_tile_candidates")
    return [(buf[2 * k], buf[2 * k + 1]) for k in range(n.value)]


def design(M: int) -> np.ndarray:
    lib = load()
    out = (c_double * (3 * M))()
    check(lib.dgfs_design(M, out), "dgfs_design")
    return np.array(out[:]).reshape(M, 3)


def interpolation_matrix(N: int, L_from: float, L_to: float) -> np.ndarray:
    """The library's one-dimensional map between species grids, [N][N]."""
    lib = load()
    out = (c_double * (N * N))()
    check(lib.dgfs_interpolation_matrix(N, float(L_from), float(L_to), out), "dgfs_interpolation_matrix")
    return np.array(out[:]).reshape(N, N)


def kernel_mode(alpha: float, gamma: float, C: float, a: float, L: float, rho: float, k, sigma) -> complex:
    """The library's host evaluation of the (VSS) kernel mode F(k, rho, sigma)."""
    lib = load()
    kk = (c_double * 3)(*[float(x) for x in k])
    sg = (c_double * 3)(*[float(x) for x in sigma])
    out = (c_double * 2)()
    check(lib.dgfs_kernel_mode(float(alpha), float(gamma), float(C), float(a), float(L), float(rho), kk, sg, out),
          "dgfs_kernel_mode")
    return complex(out[0], out[1])


def pair_tables(masses, L, N, M, n_rho, kernel, i, j, precision="f32", L_species=None) -> dict:
    """Host-side precomputed quantities of ordered pair (i, j)."""
    lib = load()
    h = _ProblemHolder(masses, L, N, M, n_rho, kernel, precision, L_species)
    info = (c_double * 6)()
    rho = (c_double * n_rho)()
    wrho = (c_double * n_rho)()
    K2 = 3 * (N // 2) ** 2 + 1
    loss = (c_double * K2)()
    check(lib.dgfs_pair_tables(ctypes.byref(h.problem), i, j, info, rho, wrho, loss), "dgfs_pair_tables")
    return {"a": info[0], "b": info[1], "gamma": info[2], "C": info[3], "R": info[4], "ndir": int(info[5]),
            "rho": np.array(rho[:]), "wrho": np.array(wrho[:]), "loss_by_k2": np.array(loss[:])}


class CollisionPlan:
    """A precomputed collision problem on the current HIP device.

    kernel[i][j] = (omega, alpha, prefactor); default: VHS with ``omega`` and the
    prefactor of eqs. (Kn)/(NVSS) with Kn0 = ``kn0``.  dealias=True evaluates eq. (sum)
    with l + m = k literally (no wrap-around; N = 16 or 32)."""

    def __init__(self, masses, N: int, L, M: int, n_rho: int, omega: float | None = None,
                 kernel=None, precision="f32", kn0: float = 1.0, tile=None, alpha: float = 1.0,
                 dealias: bool = False):
        import torch  # noqa: F401  (initialises the HIP runtime the library shares)

        if kernel is None:
            if omega is None:
                raise ValueError("give omega or kernel")
            kernel = vhs_kernel(masses, omega, alpha, kn0)
        self.masses = tuple(float(m) for m in masses)
        # L: one half-width for every species, or one per species (species-specific grids)
        Ls = np.broadcast_to(np.asarray(L, dtype=np.float64), (len(masses),))
        self.L_species = tuple(float(x) for x in Ls)
        self.s, self.N, self.L, self.M, self.n_rho = len(masses), N, max(self.L_species), M, n_rho
        self.kernel = kernel
        self.precision = _precision_code(precision)
        if tile == "auto":
            if dealias:
                tile = None   # the dealiased form runs the default geometry only
            else:
                from .autotune import best_tile
                tile = best_tile(self.masses, N, self.L_species, M, n_rho, kernel, precision)
        self.tile = tuple(tile) if tile else None
        Lsp = self.L_species if len(set(self.L_species)) > 1 else None
        self.dealias = bool(dealias)
        self._holder = _ProblemHolder(self.masses, self.L, N, M, n_rho, kernel, precision, Lsp, tile=self.tile,
                                      dealias=self.dealias)
        self._lib = load()
        handle = c_void_p()
        check(self._lib.dgfs_plan_create(ctypes.byref(self._holder.problem), ctypes.byref(handle)),
              "dgfs_plan_create")
        self._plan = handle
        self._ws = {}

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.precision == DGFS_FP64 else torch.float32

    def close(self) -> None:
        if getattr(self, "_plan", None):
            self._lib.dgfs_plan_destroy(self._plan)
            self._plan = None
        self._ws = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, batch: int) -> int:
        n = c_size_t()
        check(self._lib.dgfs_workspace_size(self._plan, batch, ctypes.byref(n)), "dgfs_workspace_size")
        return n.value

    def workspace(self, batch: int, device=None, stream=None):
        """A cached device workspace big enough for ``batch`` nodes in one pass, one per
        stream (calls on different streams may run concurrently, each needs its own).
        It is allocated on that stream, so the caching allocator orders any reuse of its
        memory after the work queued there."""
        import torch
        dev = torch.device(device or "cuda")
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        key = (str(dev), st.cuda_stream)
        need = self.workspace_bytes(batch)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < need:
            with torch.cuda.stream(st):
                ws = torch.empty(need, dtype=torch.uint8, device=dev)
            self._ws[key] = ws
        return ws

    def _check_f(self, f):
        import torch
        if not (isinstance(f, torch.Tensor) and f.is_cuda):
            raise TypeError("f must be a CUDA (HIP) tensor")
        if f.dtype != self.dtype:
            raise TypeError(f"f must be {self.dtype}")
        if not f.is_contiguous():
            raise ValueError("f must be contiguous")
        if f.dim() != 5 or tuple(f.shape[1:]) != (self.s, self.N, self.N, self.N):
            raise ValueError(f"f must be [batch][{self.s}][{self.N}][{self.N}][{self.N}]")

    def collide(self, f, out=None, pairs: bool = False, workspace=None, stream=None):
        """Q[b][i] = sum_j Q^{ij}(f[b][i], f[b][j]); with pairs=True, Q[b][i][j] = Q^{ij}."""
        import torch
        self._check_f(f)
        batch = f.shape[0]
        shape = (batch, self.s, self.s) + f.shape[2:] if pairs else tuple(f.shape)
        if out is None:
            out = torch.empty(shape, dtype=f.dtype, device=f.device)
        elif tuple(out.shape) != shape or out.dtype != f.dtype or not out.is_contiguous():
            raise ValueError("out has the wrong shape, dtype or layout")
        st = stream if stream is not None else torch.cuda.current_stream(f.device)
        ws = workspace if workspace is not None else self.workspace(max(batch, 1), f.device, st)
        if ws.data_ptr() % 256:
            raise ValueError("workspace must be 256-byte aligned")
        fn = self._lib.dgfs_collide_pairs if pairs else self._lib.dgfs_collide
        check(fn(self._plan, c_void_p(f.data_ptr()), c_void_p(out.data_ptr()), batch,
                 c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(), c_void_p(st.cuda_stream)),
              "dgfs_collide_pairs" if pairs else "dgfs_collide")
        return out

    def collide_static(self, f, out=None, stream=None):
        """collide() without a caller workspace and without any allocation in the library
        (dgfs_collide_static: the library's static device workspace, shared by every call
        on the device, so calls must not overlap).  ``out`` must be given where the caller
        cannot allocate either."""
        import torch
        self._check_f(f)
        if out is None:
            out = torch.empty(f.shape, dtype=f.dtype, device=f.device)
        elif tuple(out.shape) != tuple(f.shape) or out.dtype != f.dtype or not out.is_contiguous():
            raise ValueError("out has the wrong shape, dtype or layout")
        st = stream if stream is not None else torch.cuda.current_stream(f.device)
        check(self._lib.dgfs_collide_static(self._plan, c_void_p(f.data_ptr()), c_void_p(out.data_ptr()), f.shape[0],
                                            c_void_p(st.cuda_stream)), "dgfs_collide_static")
        return out

    def collide_timed(self, f, out=None, workspace=None, stream=None):
        """dgfs_collide with per-stage HIP-event timing (synchronous).  Returns
        (Q, stage_ms) with stage_ms = [forward FFT, gain, radial+loss, inverse FFTs, combine]."""
        import torch
        self._check_f(f)
        batch = f.shape[0]
        if out is None:
            out = torch.empty(f.shape, dtype=f.dtype, device=f.device)
        st = stream if stream is not None else torch.cuda.current_stream(f.device)
        ws = workspace if workspace is not None else self.workspace(max(batch, 1), f.device, st)
        ms = (ctypes.c_float * 5)()
        check(self._lib.dgfs_collide_timed(self._plan, c_void_p(f.data_ptr()), c_void_p(out.data_ptr()), batch,
                                           c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                           c_void_p(st.cuda_stream), ms), "dgfs_collide_timed")
        return out, list(ms)

    def collide_plain(self, f, out=None, workspace=None, stream=None):
        """The plain per-point FP64 path (dgfs_collide_plain); FP64 plans only."""
        import torch
        self._check_f(f)
        if out is None:
            out = torch.empty(f.shape, dtype=f.dtype, device=f.device)
        st = stream if stream is not None else torch.cuda.current_stream(f.device)
        ws = workspace if workspace is not None else self.workspace(1, f.device, st)
        check(self._lib.dgfs_collide_plain(self._plan, c_void_p(f.data_ptr()), c_void_p(out.data_ptr()),
                                           f.shape[0], c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                           c_void_p(st.cuda_stream)), "dgfs_collide_plain")
        return out

    def relax_step(self, f, Q, dt: float, stream=None):
        """f <- f + dt * conserve(Q) in place (one forward-Euler step), FP64 arithmetic."""
        import torch
        self._check_f(f)
        self._check_f(Q)
        st = stream if stream is not None else torch.cuda.current_stream(f.device)
        check(self._lib.dgfs_conserve_update(self._plan, c_void_p(Q.data_ptr()), c_void_p(f.data_ptr()), float(dt),
                                             f.shape[0], c_void_p(st.cuda_stream)), "dgfs_conserve_update")
        return f

    def relax_workspace_bytes(self, batch: int, scheme: str = "ssprk2") -> int:
        n = c_size_t()
        code = {"euler": _lib.DGFS_EULER, "ssprk2": _lib.DGFS_SSPRK2}[scheme]
        check(self._lib.dgfs_relax_workspace_size(self._plan, batch, code, ctypes.byref(n)),
              "dgfs_relax_workspace_size")
        return n.value

    def relax(self, f, dt: float, steps: int, scheme: str = "ssprk2", workspace=None, stream=None):
        """Advance f in place by `steps` steps of df/dt = P(Q(f)) (dgfs_relax); scheme is
        "euler" or "ssprk2" (the second-order SSP Runge-Kutta scheme)."""
        import torch
        self._check_f(f)
        code = {"euler": _lib.DGFS_EULER, "ssprk2": _lib.DGFS_SSPRK2}[scheme]
        st = stream if stream is not None else torch.cuda.current_stream(f.device)
        if workspace is None:
            # allocated on the stream that uses it: freed on return, its memory is reused
            # only by work ordered after the queued steps
            with torch.cuda.stream(st):
                workspace = torch.empty(self.relax_workspace_bytes(max(f.shape[0], 1), scheme), dtype=torch.uint8,
                                        device=f.device)
        check(self._lib.dgfs_relax(self._plan, c_void_p(f.data_ptr()), f.shape[0], float(dt), int(steps), code,
                                   c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(),
                                   c_void_p(st.cuda_stream)), "dgfs_relax")
        return f

    def conserve(self, Q, out=None, stream=None):
        """FP64 conservation projection of a raw collision result (same layout as f)."""
        import torch
        self._check_f(Q)
        if out is None:
            out = torch.empty(Q.shape, dtype=torch.float64, device=Q.device)
        st = stream if stream is not None else torch.cuda.current_stream(Q.device)
        check(self._lib.dgfs_conserve(self._plan, c_void_p(Q.data_ptr()), c_void_p(out.data_ptr()), Q.shape[0],
                                      c_void_p(st.cuda_stream)), "dgfs_conserve")
        return out


class CollisionGroup:
    """Several plans (e.g. different N) evaluated together: each plan's pipeline runs on
    its own stream forked from the caller's stream, and the whole call can be captured
    once into a hipGraph (``capture``) and replayed with a single launch."""

    def __init__(self, plans):
        self.plans = list(plans)
        self._lib = load()
        arr = (c_void_p * len(self.plans))(*[p._plan for p in self.plans])
        handle = c_void_p()
        check(self._lib.dgfs_group_create(arr, len(self.plans), ctypes.byref(handle)), "dgfs_group_create")
        self._group = handle
        self._ws = {}

    def close(self):
        if getattr(self, "_group", None):
            self._lib.dgfs_group_destroy(self._group)
            self._group = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, batches) -> int:
        b = (ctypes.c_int64 * len(self.plans))(*batches)
        n = c_size_t()
        check(self._lib.dgfs_group_workspace_size(self._group, b, ctypes.byref(n)), "dgfs_group_workspace_size")
        return n.value

    def _args(self, fs, outs, workspace, st):
        import torch
        for p, f in zip(self.plans, fs):
            p._check_f(f)
        if outs is None:
            outs = [torch.empty_like(f) for f in fs]
        batches = [f.shape[0] for f in fs]
        need = self.workspace_bytes(batches)
        ws = workspace
        if ws is None:
            # one cached workspace per calling stream, allocated on it (the group's own
            # streams fork from and join back to that stream)
            key = st.cuda_stream
            ws = self._ws.get(key)
            if ws is None or ws.numel() < need:
                with torch.cuda.stream(st):
                    ws = torch.empty(need, dtype=torch.uint8, device=fs[0].device)
                self._ws[key] = ws
        fa = (c_void_p * len(fs))(*[f.data_ptr() for f in fs])
        qa = (c_void_p * len(fs))(*[q.data_ptr() for q in outs])
        ba = (ctypes.c_int64 * len(fs))(*batches)
        return outs, ws, fa, qa, ba

    def collide(self, fs, outs=None, workspace=None, stream=None):
        import torch
        st = stream if stream is not None else torch.cuda.current_stream(fs[0].device)
        outs, ws, fa, qa, ba = self._args(fs, outs, workspace, st)
        check(self._lib.dgfs_group_collide(self._group, fa, qa, ba, c_void_p(ws.data_ptr()),
                                           ws.numel() * ws.element_size(), c_void_p(st.cuda_stream)),
              "dgfs_group_collide")
        return outs

    def capture(self, fs, outs=None, workspace=None, stream=None):
        """Capture collide(fs) into an executable graph; returns (graph, outs).  The
        buffers must stay alive and in place while the graph is used."""
        import torch
        st = stream if stream is not None else torch.cuda.Stream(fs[0].device)
        outs, ws, fa, qa, ba = self._args(fs, outs, workspace, st)
        g = c_void_p()
        check(self._lib.dgfs_group_capture(self._group, fa, qa, ba, c_void_p(ws.data_ptr()),
                                           ws.numel() * ws.element_size(), c_void_p(st.cuda_stream),
                                           ctypes.byref(g)), "dgfs_group_capture")
        return Graph(self._lib, g, st, keep=(fs, outs, ws)), outs


class Graph:
    """An instantiated hipGraph of a group call."""

    def __init__(self, lib, handle, stream, keep):
        self._lib, self._g, self.stream, self._keep = lib, handle, stream, keep

    def launch(self, stream=None):
        st = stream if stream is not None else self.stream
        check(self._lib.dgfs_graph_launch(self._g, c_void_p(st.cuda_stream)), "dgfs_graph_launch")

    def close(self):
        if getattr(self, "_g", None):
            self._lib.dgfs_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def slab_gll(K: int):
    """The library's GLL points and weights on [-1, 1]."""
    lib = load()
    x = (c_double * K)()
    w = (c_double * K)()
    check(lib.dgfs_slab_gll(K, x, w), "dgfs_slab_gll")
    return np.array(x[:]), np.array(w[:])


def _boundary(spec: dict, s: int) -> "_lib.Boundary":
    b = _lib.Boundary()
    b.kind = {"inflow": _lib.DGFS_BC_INFLOW, "wall": _lib.DGFS_BC_WALL}[spec["kind"]]
    n = list(spec.get("n", ())) + [0.0] * (8 - len(spec.get("n", ())))
    b.n = (c_double * 8)(*n[:8])
    b.u = (c_double * 3)(*[float(x) for x in spec.get("u", (0.0, 0.0, 0.0))])
    b.T = float(spec["T"])
    return b


class Slab:
    """1-D slab of Ne elements x K GLL nodes around a CollisionPlan (dgfs_slab_*).
    left/right: {"kind": "inflow", "n": (n_1, ..., n_s), "u": (ux, uy, uz), "T": T} or
    {"kind": "wall", "u": (0, uy, uz), "T": T} (purely diffuse).  The state is a tensor
    [Ne*K][s][N][N][N] of the plan's dtype, node e*K + m."""

    def __init__(self, plan: "CollisionPlan", x0: float, x1: float, Ne: int, K: int, left: dict, right: dict,
                 collide: bool = True):
        self.plan, self.Ne, self.K = plan, Ne, K
        self._lib = load()
        d = _lib.SlabDesc()
        d.x0, d.x1, d.Ne, d.K = float(x0), float(x1), int(Ne), int(K)
        d.left, d.right = _boundary(left, plan.s), _boundary(right, plan.s)
        d.collide = 1 if collide else 0
        handle = c_void_p()
        check(self._lib.dgfs_slab_create(plan._plan, ctypes.byref(d), ctypes.byref(handle)), "dgfs_slab_create")
        self._slab = handle

    def workspace_bytes(self, scheme: str = "ssprk2") -> int:
        n = c_size_t()
        code = {"euler": _lib.DGFS_EULER, "ssprk2": _lib.DGFS_SSPRK2}[scheme]
        check(self._lib.dgfs_slab_workspace_size(self._slab, code, ctypes.byref(n)), "dgfs_slab_workspace_size")
        return n.value

    def step(self, f, dt: float, steps: int = 1, scheme: str = "ssprk2", workspace=None, stream=None):
        import torch
        if f.dim() != 5 or f.shape[0] != self.Ne * self.K:
            raise ValueError("f must be [Ne*K][s][N][N][N]")
        self.plan._check_f(f)
        code = {"euler": _lib.DGFS_EULER, "ssprk2": _lib.DGFS_SSPRK2}[scheme]
        st = stream if stream is not None else torch.cuda.current_stream(f.device)
        if workspace is None:
            with torch.cuda.stream(st):   # see CollisionPlan.relax
                workspace = torch.empty(self.workspace_bytes(scheme), dtype=torch.uint8, device=f.device)
        check(self._lib.dgfs_slab_step(self._slab, c_void_p(f.data_ptr()), float(dt), int(steps), code,
                                       c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(),
                                       c_void_p(st.cuda_stream)), "dgfs_slab_step")
        return f

    def close(self):
        if getattr(self, "_slab", None):
            self._lib.dgfs_slab_destroy(self._slab)
            self._slab = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
