"""ctypes binding of libdgfs.so (the C ABI declared in include/dgfs.h).

Argument marshalling only: every step of the collision operator runs in the HIP
kernels of the library.  Importing this module without a built library raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_size_t, c_void_p

LIB_PATH = os.environ.get("DGFS_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                          "libdgfs.so")

DGFS_OK, DGFS_EINVAL, DGFS_EUNSUPPORTED, DGFS_ENOMEM, DGFS_EDEVICE = 0, -1, -2, -3, -4
DGFS_FP32, DGFS_FP64 = 0, 1

EXPORTED = (
    "dgfs_check_problem", "dgfs_pair_prefactor", "dgfs_plan_create", "dgfs_plan_destroy", "dgfs_workspace_size",
    "dgfs_collide", "dgfs_collide_static", "dgfs_static_workspace_bytes", "dgfs_collide_timed", "dgfs_collide_pairs", "dgfs_collide_plain", "dgfs_conserve",
    "dgfs_conserve_update", "dgfs_pair_tables", "dgfs_design", "dgfs_interpolation_matrix", "dgfs_kernel_mode",
    "dgfs_status_string", "dgfs_last_error", "dgfs_tile_candidates", "dgfs_group_create", "dgfs_group_destroy",
    "dgfs_group_workspace_size", "dgfs_group_collide", "dgfs_group_capture", "dgfs_graph_launch",
    "dgfs_graph_destroy", "dgfs_probe_valu", "dgfs_relax_workspace_size", "dgfs_relax",
    "dgfs_slab_create", "dgfs_slab_destroy", "dgfs_slab_workspace_size", "dgfs_slab_step", "dgfs_slab_gll",
)

DGFS_BC_INFLOW, DGFS_BC_WALL = 0, 1

DGFS_EULER, DGFS_SSPRK2 = 0, 1


class PairKernel(ctypes.Structure):
    _fields_ = [("omega", c_double), ("alpha", c_double), ("prefactor", c_double)]


class Problem(ctypes.Structure):
    _fields_ = [
        ("s", c_int32),
        ("mass", POINTER(c_double)),
        ("L", c_double),
        ("L_species", POINTER(c_double)),
        ("N", c_int32),
        ("M", c_int32),
        ("n_rho", c_int32),
        ("kernel", POINTER(PairKernel)),
        ("precision", c_int32),
        ("tile_ch", c_int32),
        ("tile_cz", c_int32),
        ("dealias", c_int32),
    ]


class Boundary(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("n", c_double * 8), ("u", c_double * 3), ("T", c_double)]


class SlabDesc(ctypes.Structure):
    _fields_ = [("x0", c_double), ("x1", c_double), ("Ne", c_int32), ("K", c_int32),
                ("left", Boundary), ("right", Boundary), ("collide", c_int32)]


class DgfsError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load libdgfs.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1903_03056_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    lib.dgfs_check_problem.argtypes = [POINTER(Problem)]
    lib.dgfs_pair_prefactor.argtypes = [c_double, c_double, c_double, c_double, c_double, POINTER(c_double)]
    lib.dgfs_plan_create.argtypes = [POINTER(Problem), POINTER(c_void_p)]
    lib.dgfs_plan_destroy.argtypes = [c_void_p]
    lib.dgfs_plan_destroy.restype = None
    lib.dgfs_workspace_size.argtypes = [c_void_p, c_int64, POINTER(c_size_t)]
    for name in ("dgfs_collide", "dgfs_collide_pairs", "dgfs_collide_plain"):
        getattr(lib, name).argtypes = [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_size_t, c_void_p]
    lib.dgfs_collide_timed.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_size_t, c_void_p,
                                       POINTER(ctypes.c_float)]
    lib.dgfs_collide_static.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, c_void_p]
    lib.dgfs_static_workspace_bytes.argtypes = []
    lib.dgfs_static_workspace_bytes.restype = c_size_t
    lib.dgfs_conserve.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, c_void_p]
    lib.dgfs_conserve_update.argtypes = [c_void_p, c_void_p, c_void_p, c_double, c_int64, c_void_p]
    lib.dgfs_pair_tables.argtypes = [POINTER(Problem), c_int32, c_int32, POINTER(c_double), POINTER(c_double),
                                     POINTER(c_double), POINTER(c_double)]
    lib.dgfs_design.argtypes = [c_int32, POINTER(c_double)]
    lib.dgfs_interpolation_matrix.argtypes = [c_int32, c_double, c_double, POINTER(c_double)]
    lib.dgfs_kernel_mode.argtypes = [c_double, c_double, c_double, c_double, c_double, c_double, POINTER(c_double),
                                     POINTER(c_double), POINTER(c_double)]
    lib.dgfs_probe_valu.argtypes = [c_void_p, c_size_t, c_int32, c_int32, c_void_p, POINTER(c_double)]
    lib.dgfs_relax_workspace_size.argtypes = [c_void_p, c_int64, c_int32, POINTER(c_size_t)]
    lib.dgfs_relax.argtypes = [c_void_p, c_void_p, c_int64, c_double, c_int32, c_int32, c_void_p, c_size_t, c_void_p]
    lib.dgfs_slab_create.argtypes = [c_void_p, POINTER(SlabDesc), POINTER(c_void_p)]
    lib.dgfs_slab_destroy.argtypes = [c_void_p]
    lib.dgfs_slab_destroy.restype = None
    lib.dgfs_slab_workspace_size.argtypes = [c_void_p, c_int32, POINTER(c_size_t)]
    lib.dgfs_slab_step.argtypes = [c_void_p, c_void_p, c_double, c_int32, c_int32, c_void_p, c_size_t, c_void_p]
    lib.dgfs_slab_gll.argtypes = [c_int32, POINTER(c_double), POINTER(c_double)]
    lib.dgfs_tile_candidates.argtypes = [c_int32, c_int32, POINTER(c_int32), c_int32, POINTER(c_int32)]
    lib.dgfs_group_create.argtypes = [POINTER(c_void_p), c_int32, POINTER(c_void_p)]
    lib.dgfs_group_destroy.argtypes = [c_void_p]
    lib.dgfs_group_destroy.restype = None
    lib.dgfs_group_workspace_size.argtypes = [c_void_p, POINTER(c_int64), POINTER(c_size_t)]
    lib.dgfs_group_collide.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_int64), c_void_p,
                                       c_size_t, c_void_p]
    lib.dgfs_group_capture.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_int64), c_void_p,
                                       c_size_t, c_void_p, POINTER(c_void_p)]
    lib.dgfs_graph_launch.argtypes = [c_void_p, c_void_p]
    lib.dgfs_graph_destroy.argtypes = [c_void_p]
    lib.dgfs_graph_destroy.restype = None
    lib.dgfs_status_string.argtypes = [c_int32]
    lib.dgfs_status_string.restype = ctypes.c_char_p
    lib.dgfs_last_error.argtypes = []
    lib.dgfs_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("dgfs_plan_destroy", "dgfs_status_string", "dgfs_last_error", "dgfs_group_destroy",
                        "dgfs_graph_destroy", "dgfs_slab_destroy", "dgfs_static_workspace_bytes"):
            getattr(lib, name).restype = c_int32
    _lib = lib
    return lib


def check(status: int, where: str) -> None:
    if status != DGFS_OK:
        lib = load()
        raise DgfsError(status, where, lib.dgfs_last_error().decode())
