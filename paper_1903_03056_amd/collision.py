"""Python face of the collision library: plan creation and the collide / conserve calls.

PyTorch supplies device memory and streams; the arithmetic runs in libdgfs.so.
"""
from __future__ import annotations

import ctypes
import math
from ctypes import POINTER, c_double, c_size_t, c_void_p

import numpy as np

from . import _lib
from ._lib import DGFS_FP32, DGFS_FP64, PairKernel, Problem, check, load


def vhs_prefactor(mi: float, mj: float, omega: float, alpha: float = 1.0, kn0: float = 1.0) -> float:
    """Kn_ij^{-1} times the constant of the dimensionless VSS kernel (Sec. 3, eqs. Kn
    and NVSS).  The sqrt(1 + m_i/m_j) factors of the two cancel, leaving
    alpha / (Kn0 2^{1+alpha} Gamma(5/2 - omega) pi mu_ij^{omega - 1/2}), mu_ij the reduced mass."""
    mu = mi * mj / (mi + mj)
    return alpha / (kn0 * 2.0 ** (1.0 + alpha) * math.gamma(2.5 - omega) * math.pi * mu ** (omega - 0.5))


def _precision_code(precision) -> int:
    if precision in ("f32", "fp32", "float32", DGFS_FP32):
        return DGFS_FP32
    if precision in ("f64", "fp64", "float64", DGFS_FP64):
        return DGFS_FP64
    raise ValueError(f"unknown precision {precision!r}")


class _ProblemHolder:
    """Keeps the ctypes arrays alive as long as the Problem struct refers to them."""

    def __init__(self, masses, L, N, M, n_rho, kernel, precision, L_species=None):
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
                               N=N, M=M, n_rho=n_rho, kernel=self.kern, precision=_precision_code(precision))


def vhs_kernel(masses, omega, alpha: float = 1.0, kn0: float = 1.0):
    s = len(masses)
    return [[(omega, alpha, vhs_prefactor(masses[i], masses[j], omega, alpha, kn0)) for j in range(s)]
            for i in range(s)]


def check_problem(masses, L, N, M, n_rho, kernel, precision="f32", L_species=None) -> int:
    """Host-side validation; returns the dgfs status code (0 = ok)."""
    h = _ProblemHolder(masses, L, N, M, n_rho, kernel, precision, L_species)
    return load().dgfs_check_problem(ctypes.byref(h.problem))


def design(M: int) -> np.ndarray:
    lib = load()
    out = (c_double * (3 * M))()
    check(lib.dgfs_design(M, out), "dgfs_design")
    return np.array(out[:]).reshape(M, 3)


def pair_tables(masses, L, N, M, n_rho, kernel, i, j, precision="f32") -> dict:
    """Host-side precomputed quantities of ordered pair (i, j)."""
    lib = load()
    h = _ProblemHolder(masses, L, N, M, n_rho, kernel, precision)
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
    prefactor of eqs. (Kn)/(NVSS) with Kn0 = ``kn0``."""

    def __init__(self, masses, N: int, L: float, M: int, n_rho: int, omega: float | None = None,
                 kernel=None, precision="f32", kn0: float = 1.0):
        import torch  # noqa: F401  (initialises the HIP runtime the library shares)

        if kernel is None:
            if omega is None:
                raise ValueError("give omega or kernel")
            kernel = vhs_kernel(masses, omega, 1.0, kn0)
        self.masses = tuple(float(m) for m in masses)
        self.s, self.N, self.L, self.M, self.n_rho = len(masses), N, float(L), M, n_rho
        self.kernel = kernel
        self.precision = _precision_code(precision)
        self._holder = _ProblemHolder(self.masses, L, N, M, n_rho, kernel, precision)
        self._lib = load()
        handle = c_void_p()
        check(self._lib.dgfs_plan_create(ctypes.byref(self._holder.problem), ctypes.byref(handle)),
              "dgfs_plan_create")
        self._plan = handle
        self._ws = None

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.precision == DGFS_FP64 else torch.float32

    def close(self) -> None:
        if getattr(self, "_plan", None):
            self._lib.dgfs_plan_destroy(self._plan)
            self._plan = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, batch: int) -> int:
        n = c_size_t()
        check(self._lib.dgfs_workspace_size(self._plan, batch, ctypes.byref(n)), "dgfs_workspace_size")
        return n.value

    def workspace(self, batch: int, device=None):
        """A cached device workspace big enough for ``batch`` nodes in one pass."""
        import torch
        need = self.workspace_bytes(batch)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=device or "cuda")
        return self._ws

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
        ws = workspace if workspace is not None else self.workspace(max(batch, 1), f.device)
        if ws.data_ptr() % 256:
            raise ValueError("workspace must be 256-byte aligned")
        st = stream if stream is not None else torch.cuda.current_stream(f.device)
        fn = self._lib.dgfs_collide_pairs if pairs else self._lib.dgfs_collide
        check(fn(self._plan, c_void_p(f.data_ptr()), c_void_p(out.data_ptr()), batch,
                 c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(), c_void_p(st.cuda_stream)),
              "dgfs_collide_pairs" if pairs else "dgfs_collide")
        return out

    def collide_timed(self, f, out=None, workspace=None, stream=None):
        """dgfs_collide with per-stage HIP-event timing (synchronous).  Returns
        (Q, stage_ms) with stage_ms = [forward FFT, gain, radial+loss, inverse FFTs, combine]."""
        import torch
        self._check_f(f)
        batch = f.shape[0]
        if out is None:
            out = torch.empty(f.shape, dtype=f.dtype, device=f.device)
        ws = workspace if workspace is not None else self.workspace(max(batch, 1), f.device)
        st = stream if stream is not None else torch.cuda.current_stream(f.device)
        ms = (ctypes.c_float * 5)()
        check(self._lib.dgfs_collide_timed(self._plan, c_void_p(f.data_ptr()), c_void_p(out.data_ptr()), batch,
                                           c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                           c_void_p(st.cuda_stream), ms), "dgfs_collide_timed")
        return out, list(ms)

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
