"""ctypes mirror of include/trmc.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

from . import build as _build

HOMOG, SLAB1D = 1, 2
FP64, FP32_MIXED = 1, 2
NATURAL, FIXED, ADAPTIVE, ADAPTIVE_REUSE = 0, 1, 2, 3
WB_OFF, WB_MIN, WB_MEAN = 0, 1, 2
BC_SPECULAR, BC_INFLOW = 0, 1
MAJORANT_STEP, MAJORANT_LEVEL = 0, 1

EINVAL, ENOMEM, ENOSPC, EIO, EOVERFLOW, EBUSY = -22, -12, -28, -5, -75, -16
CELL_OVERFLOW = 1

EXPORTS = [
    "trmc_abi_version", "trmc_strerror", "trmc_workspace_size", "trmc_ctx_workspace_size", "trmc_init",
    "trmc_step", "trmc_moments", "trmc_state", "trmc_read", "trmc_admit", "trmc_retire", "trmc_sync",
    "trmc_destroy", "trmc_set_schedule", "trmc_get_schedule", "trmc_use_graph", "trmc_count",
    "trmc_fuse_steps", "trmc_moments_async", "trmc_order_by_cost", "trmc_step_static",
    "trmc_set_budget",
]

SCHED_BUCKETS = 32
PATH_DEFAULT, PATH_GROUP, PATH_WAVE, PATH_TILED = 0, 1, 2, 3


class Desc(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("seed", ctypes.c_uint32), ("uid", ctypes.c_uint32),
        ("geometry", ctypes.c_uint32), ("n_particles", ctypes.c_uint64), ("n_cells", ctypes.c_uint32),
        ("precision", ctypes.c_uint32), ("length", ctypes.c_double), ("dt", ctypes.c_double),
        ("particle_weight", ctypes.c_double), ("eps", ctypes.c_double),
        ("eps_cells", ctypes.POINTER(ctypes.c_double)), ("alpha", ctypes.c_double),
        ("trunc", ctypes.c_uint32), ("m_init", ctypes.c_uint32), ("m_cap", ctypes.c_uint32),
        ("step0", ctypes.c_uint32), ("delta1", ctypes.c_double), ("delta2", ctypes.c_double),
        ("m_state0", ctypes.POINTER(ctypes.c_uint32)),
        ("wb", ctypes.c_uint32), ("wb_mmax", ctypes.c_uint32),
        ("bc", ctypes.c_uint32), ("n_live0", ctypes.c_uint32),
        ("in_left", ctypes.c_double * 3), ("in_right", ctypes.c_double * 3),
        ("majorant", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
    ]


class Particles(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("vx", ctypes.c_void_p), ("vy", ctypes.c_void_p),
                ("vz", ctypes.c_void_p)]


class CellMoments(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint32), ("m_state", ctypes.c_uint32),
        ("rho", ctypes.c_double), ("ux", ctypes.c_double), ("uy", ctypes.c_double), ("uz", ctypes.c_double),
        ("T", ctypes.c_double), ("Pxx", ctypes.c_double), ("Pyy", ctypes.c_double), ("Pzz", ctypes.c_double),
        ("M4", ctypes.c_double),
        ("collisions", ctypes.c_uint64), ("dummies", ctypes.c_uint64), ("violations", ctypes.c_uint64),
        ("work_collisions", ctypes.c_uint64),
        ("thermalized", ctypes.c_uint32), ("borrowed", ctypes.c_uint32), ("m_eff", ctypes.c_uint32),
        ("m_used", ctypes.c_uint32), ("attempts", ctypes.c_uint32), ("N0", ctypes.c_uint32),
        ("R0", ctypes.c_uint32), ("status", ctypes.c_uint32), ("wb_thermalized", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32), ("q", ctypes.c_double), ("g", ctypes.c_double),
    ]


_lib = None


def lib_path() -> str:
    return _build.LIB


def load():
    """Load the in-tree libtrmc.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it first (python -m paper_1009_2768_amd.build)")
    # torch ships its own HIP runtime under the same soname as ROCm's: load it
    # first, so that the library binds to the runtime that owns torch's device
    # memory and streams (loaded the other way round, two runtimes coexist and
    # the library's copies of torch tensors fail)
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp, u32, sz, i = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_size_t, ctypes.c_int
    L.trmc_abi_version.argtypes = []
    L.trmc_abi_version.restype = i
    L.trmc_strerror.argtypes = [i]
    L.trmc_strerror.restype = ctypes.c_char_p
    L.trmc_workspace_size.argtypes = [P(Desc), u32, P(sz)]
    L.trmc_workspace_size.restype = i
    L.trmc_ctx_workspace_size.argtypes = [u32, u32, P(sz)]
    L.trmc_ctx_workspace_size.restype = i
    L.trmc_init.argtypes = [P(vp), P(Desc), u32, P(Particles), vp, sz, u32, u32, vp]
    L.trmc_init.restype = i
    L.trmc_step.argtypes = [vp, u32]
    L.trmc_step.restype = i
    L.trmc_moments.argtypes = [vp, u32, P(CellMoments), u32]
    L.trmc_moments.restype = i
    L.trmc_state.argtypes = [vp, u32, P(Particles)]
    L.trmc_state.restype = i
    L.trmc_read.argtypes = [vp, u32, vp, vp, vp, vp, P(u32), P(u32)]
    L.trmc_read.restype = i
    L.trmc_admit.argtypes = [vp, P(Desc), P(Particles), vp, sz, P(u32)]
    L.trmc_admit.restype = i
    L.trmc_retire.argtypes = [vp, u32]
    L.trmc_retire.restype = i
    L.trmc_sync.argtypes = [vp]
    L.trmc_sync.restype = i
    L.trmc_destroy.argtypes = [vp]
    L.trmc_destroy.restype = i
    L.trmc_set_schedule.argtypes = [vp, P(u32), u32]
    L.trmc_set_schedule.restype = i
    L.trmc_get_schedule.argtypes = [vp, P(u32), u32]
    L.trmc_get_schedule.restype = i
    L.trmc_use_graph.argtypes = [vp, i]
    L.trmc_use_graph.restype = i
    L.trmc_fuse_steps.argtypes = [vp, i]
    L.trmc_fuse_steps.restype = i
    L.trmc_order_by_cost.argtypes = [vp, i]
    L.trmc_order_by_cost.restype = i
    L.trmc_step_static.argtypes = [P(Desc), P(Particles), u32, vp]
    L.trmc_step_static.restype = i
    L.trmc_set_budget.argtypes = [vp, ctypes.c_uint64]
    L.trmc_set_budget.restype = i
    L.trmc_moments_async.argtypes = [vp, u32, vp, u32]
    L.trmc_moments_async.restype = i
    L.trmc_count.argtypes = [vp, u32, P(ctypes.c_uint64)]
    L.trmc_count.restype = i
    _lib = L
    return L


class TrmcError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        msg = load().trmc_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})")


def check(code: int, what: str):
    if code != 0:
        raise TrmcError(code, what)
