"""MI355X (gfx950) TRMC-R: Python binding of libtrmc.

The library implements the recursive time-relaxed Monte Carlo collision step of
Trazzi, Pareschi and Wennberg (Wild-sum split, recursive collision trees with
twin reuse, VHS dummy collisions, conservative Maxwellian remainder, adaptive
depth), fused with slab transport and a stable counting sort, in hand-written HIP
kernels behind the C ABI of include/trmc.h.  This module only marshals
arguments: PyTorch provides device memory and the stream; every step of the
method runs in the library's kernels.  There is no CPU path.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np

from . import _abi
from ._abi import (ADAPTIVE, ADAPTIVE_REUSE, FIXED, FP32_MIXED, FP64, HOMOG, NATURAL, PATH_DEFAULT, PATH_GROUP, PATH_TILED,
                   PATH_WAVE, SCHED_BUCKETS, SLAB1D, WB_MEAN, WB_MIN, WB_OFF, BC_INFLOW, BC_SPECULAR, MAJORANT_LEVEL,
                   MAJORANT_STEP, TrmcError, check)

__all__ = ["Instance", "Context", "HOMOG", "SLAB1D", "FP64", "FP32_MIXED", "NATURAL", "FIXED", "ADAPTIVE",
           "ADAPTIVE_REUSE",
           "PATH_DEFAULT", "PATH_GROUP", "PATH_WAVE", "PATH_TILED", "SCHED_BUCKETS", "WB_OFF", "WB_MIN",
           "WB_MEAN", "BC_SPECULAR", "BC_INFLOW", "MAJORANT_STEP", "MAJORANT_LEVEL", "TrmcError", "load", "size_bucket", "moments_record_bytes",
           "unpack_moments"]

load = _abi.load


@dataclass
class Instance:
    """Parameters of one homogeneous solve or 1-D slab (mirrors trmc_desc)."""
    n_particles: int
    geometry: int = HOMOG
    n_cells: int = 1
    precision: int = FP64
    seed: int = 0
    uid: int = 0
    length: float = 1.0
    dt: float = 0.05
    particle_weight: float | None = None
    eps: float = 1.0
    eps_cells: np.ndarray | None = None
    alpha: float = 0.0
    trunc: int = NATURAL
    m_init: int = 2
    m_cap: int = 64
    step0: int = 0
    delta1: float = 0.005
    delta2: float = 0.01
    m_state0: np.ndarray | None = None
    wb: int = WB_OFF  # tree-shape truncation (Sec. 4.4): WB_MIN (def:2) or WB_MEAN (def:3)
    wb_mmax: int = 5
    bc: int = BC_SPECULAR  # BC_INFLOW: open slab with reservoirs (n_particles is then the capacity)
    n_live0: int = 0       # open slab: particles present at admission
    in_left: tuple | None = None   # reservoir (rho, u, T) at x = 0
    in_right: tuple | None = None  # reservoir (rho, u, T) at x = length
    majorant: int = MAJORANT_STEP  # MAJORANT_LEVEL: VHS bound raised level by level (Remark 4.1)
    _keep: list = field(default_factory=list, repr=False)

    def to_c(self) -> _abi.Desc:
        d = _abi.Desc()
        d.struct_size = ctypes.sizeof(_abi.Desc)
        d.seed, d.uid, d.geometry = self.seed, self.uid, self.geometry
        d.n_particles, d.n_cells, d.precision = self.n_particles, self.n_cells, self.precision
        d.length, d.dt = self.length, self.dt
        w = self.particle_weight
        if w is None:
            w = self.length / max(1, self.n_particles)
        d.particle_weight = w
        d.eps, d.alpha = self.eps, self.alpha
        d.trunc, d.m_init, d.m_cap, d.step0 = self.trunc, self.m_init, self.m_cap, self.step0
        d.delta1, d.delta2 = self.delta1, self.delta2
        d.wb, d.wb_mmax = self.wb, self.wb_mmax
        d.bc, d.n_live0 = self.bc, self.n_live0
        d.majorant = self.majorant
        if self.in_left is not None:
            d.in_left = (ctypes.c_double * 3)(*self.in_left)
        if self.in_right is not None:
            d.in_right = (ctypes.c_double * 3)(*self.in_right)
        self._keep = []
        if self.eps_cells is not None:
            e = np.ascontiguousarray(self.eps_cells, dtype=np.float64)
            self._keep.append(e)
            d.eps_cells = e.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if self.m_state0 is not None:
            m = np.ascontiguousarray(self.m_state0, dtype=np.uint32)
            self._keep.append(m)
            d.m_state0 = m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
        return d

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.precision == FP64 else torch.float32

    @property
    def np_dtype(self):
        return np.float64 if self.precision == FP64 else np.float32


def size_bucket(inst: Instance) -> int:
    """Schedule bucket of an instance's cells: floor(log2) of the expected particles
    per cell (the rule of trmc_set_schedule)."""
    per = inst.n_particles / (inst.n_cells if inst.geometry == SLAB1D else 1)
    b = 0
    while b + 1 < SCHED_BUCKETS and per >= float(2 << b):
        b += 1
    return b


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream), stream


def _particles(t: dict) -> _abi.Particles:
    p = _abi.Particles()
    p.x = t["x"].data_ptr() if t.get("x") is not None else None
    p.vx, p.vy, p.vz = t["vx"].data_ptr(), t["vy"].data_ptr(), t["vz"].data_ptr()
    return p


def moments_record_bytes(n_cells: int) -> int:
    """Bytes of the records of n_cells cells written by Context.moments_async."""
    return n_cells * ctypes.sizeof(_abi.CellMoments)


def unpack_moments(buf, n_cells: int) -> dict:
    """The dict of Context.moments from a host uint8 tensor (or array) filled by
    Context.moments_async."""
    raw = buf.numpy() if hasattr(buf, "numpy") else np.asarray(buf)
    rec = raw[: moments_record_bytes(n_cells)].view(np.dtype(_abi.CellMoments))
    return {k: np.array(rec[k]) for k in rec.dtype.names}


class Context:
    """A set of instances stepped together on one HIP stream.

    ``particles[i]`` is a dict of device tensors ``x`` (slab only), ``vx``, ``vy``,
    ``vz`` of the instance's precision; the tensors are kept alive by the context.
    """

    def __init__(self, instances, particles, max_instances=None, max_cells=None, stream=None, device="cuda"):
        import torch
        L = _abi.load()
        if not torch.cuda.is_available():
            raise RuntimeError("libtrmc needs a ROCm GPU; none is visible")
        self._lib = L
        self.device = torch.device(device)
        self.instances = list(instances)
        n = len(self.instances)
        self.max_instances = max_instances or max(1, n)
        cells = sum(i.n_cells if i.geometry == SLAB1D else 1 for i in self.instances)
        self.max_cells = max_cells or max(1, cells)
        descs = (_abi.Desc * max(1, n))()
        bufs = (_abi.Particles * max(1, n))()
        for k, (inst, t) in enumerate(zip(self.instances, particles)):
            descs[k] = inst.to_c()
            bufs[k] = _particles(t)
        self._descs = descs
        self._bufs = bufs
        self._particles = list(particles)
        ws = ctypes.c_size_t(0)
        cws = ctypes.c_size_t(0)
        check(L.trmc_workspace_size(descs, n, ctypes.byref(ws)), "trmc_workspace_size")
        check(L.trmc_ctx_workspace_size(self.max_instances, self.max_cells, ctypes.byref(cws)),
              "trmc_ctx_workspace_size")
        total = ws.value + cws.value
        self.workspace = torch.empty(max(total, 256) + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_off = (-base) % 256
        self._handle, self.stream = _stream_handle(stream)
        ctx = ctypes.c_void_p()
        check(L.trmc_init(ctypes.byref(ctx), descs, n, bufs, ctypes.c_void_p(base + self._ws_off), total,
                          self.max_instances, self.max_cells, self._handle), "trmc_init")
        self._ctx = ctx
        self._admitted = {k: (inst, particles[k], None) for k, inst in enumerate(self.instances)}

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.trmc_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stepping ----------------------------------------------------------
    def step(self, n: int = 1):
        check(self._lib.trmc_step(self._ctx, n), "trmc_step")

    def sync(self):
        check(self._lib.trmc_sync(self._ctx), "trmc_sync")

    # -- batching ----------------------------------------------------------
    def set_schedule(self, paths):
        """Kernel path per size bucket (list of PATH_* values, at most SCHED_BUCKETS)."""
        a = (ctypes.c_uint32 * max(1, len(paths)))(*[int(p) for p in paths])
        check(self._lib.trmc_set_schedule(self._ctx, a, len(paths)), "trmc_set_schedule")

    def get_schedule(self):
        a = (ctypes.c_uint32 * SCHED_BUCKETS)()
        check(self._lib.trmc_get_schedule(self._ctx, a, SCHED_BUCKETS), "trmc_get_schedule")
        return list(a)

    def use_graph(self, on: bool = True):
        """Replay one captured HIP graph per step instead of launching each kernel."""
        check(self._lib.trmc_use_graph(self._ctx, 1 if on else 0), "trmc_use_graph")

    def order_by_cost(self, on: bool = True):
        """Sort the whole-cell work lists by each cell's last measured step time before
        every launch, longest first (the default); off: the order of expected size."""
        check(self._lib.trmc_order_by_cost(self._ctx, 1 if on else 0), "trmc_order_by_cost")

    def fuse_steps(self, on: bool = True):
        """Let step(n) take homogeneous cells through all n steps in one launch (the default)."""
        check(self._lib.trmc_fuse_steps(self._ctx, 1 if on else 0), "trmc_fuse_steps")

    # -- serving -----------------------------------------------------------
    def admit(self, inst: Instance, particles: dict) -> int:
        import torch
        L = self._lib
        d = inst.to_c()
        ws = ctypes.c_size_t(0)
        check(L.trmc_workspace_size(ctypes.byref(d), 1, ctypes.byref(ws)), "trmc_workspace_size")
        buf = torch.empty(ws.value + 256, dtype=torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        p = _particles(particles)
        slot = ctypes.c_uint32(0)
        check(L.trmc_admit(self._ctx, ctypes.byref(d), ctypes.byref(p), ctypes.c_void_p(buf.data_ptr() + off),
                           ws.value, ctypes.byref(slot)), "trmc_admit")
        self._admitted[slot.value] = (inst, particles, buf)
        return slot.value

    def set_budget(self, nbytes: int):
        """Device memory (workspaces and particle arrays) the active instances may
        occupy; admit() raises TrmcError with code EBUSY beyond it (0: no budget)."""
        check(self._lib.trmc_set_budget(self._ctx, int(nbytes)), "trmc_set_budget")

    def retire(self, slot: int):
        check(self._lib.trmc_retire(self._ctx, slot), "trmc_retire")
        self._admitted.pop(slot, None)

    def instance(self, slot: int) -> Instance:
        return self._admitted[slot][0]

    # -- results -----------------------------------------------------------
    def moments(self, slot: int):
        inst = self.instance(slot)
        nc = inst.n_cells if inst.geometry == SLAB1D else 1
        out = (_abi.CellMoments * nc)()
        check(self._lib.trmc_moments(self._ctx, slot, out, nc), "trmc_moments")
        names = [f[0] for f in _abi.CellMoments._fields_]
        return {k: np.array([getattr(out[c], k) for c in range(nc)]) for k in names}

    def moments_async(self, slot: int, out) -> None:
        """Enqueue the moments of `slot` into `out`, a pinned host (or device) uint8
        tensor of at least n_cells records (moments_record_bytes); the contents are
        valid once the context's stream has passed this call.  unpack_moments
        turns them into the dict of moments()."""
        cap = (out.numel() * out.element_size()) // ctypes.sizeof(_abi.CellMoments)
        check(self._lib.trmc_moments_async(self._ctx, slot, ctypes.c_void_p(out.data_ptr()), cap),
              "trmc_moments_async")

    def read(self, slot: int):
        inst = self.instance(slot)
        n = inst.n_particles
        nc = inst.n_cells if inst.geometry == SLAB1D else 1
        dt = inst.np_dtype
        x = np.zeros(n, dtype=dt) if inst.geometry == SLAB1D else None
        vx, vy, vz = np.zeros(n, dtype=dt), np.zeros(n, dtype=dt), np.zeros(n, dtype=dt)
        ms = np.zeros(nc, dtype=np.uint32)
        step = ctypes.c_uint32(0)
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a is not None else None  # noqa: E731
        check(self._lib.trmc_read(self._ctx, slot, ptr(x), ptr(vx), ptr(vy), ptr(vz),
                                  ms.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), ctypes.byref(step)),
              "trmc_read")
        live = self.count(slot)
        if live != n:
            x = x[:live] if x is not None else None
            vx, vy, vz = vx[:live], vy[:live], vz[:live]
        return {"x": x, "vx": vx, "vy": vy, "vz": vz, "m_state": ms, "step": step.value}

    def count(self, slot: int) -> int:
        """Particles of instance `slot` now (an open slab's count changes every step)."""
        n = ctypes.c_uint64(0)
        check(self._lib.trmc_count(self._ctx, slot, ctypes.byref(n)), "trmc_count")
        return int(n.value)

    def state_pointers(self, slot: int):
        p = _abi.Particles()
        check(self._lib.trmc_state(self._ctx, slot, ctypes.byref(p)), "trmc_state")
        return p


def device_particles(vx, vy, vz, x=None, precision=FP64, device="cuda", capacity=None):
    """Copy host arrays to device tensors of the instance precision (zero-padded to
    `capacity` elements for an open slab)."""
    import torch
    dt = torch.float64 if precision == FP64 else torch.float32
    n = len(vx)
    cap = max(n, capacity or 0)

    def dev(a):
        b = np.zeros(cap)
        b[:n] = np.asarray(a, dtype=np.float64)
        return torch.as_tensor(b, dtype=dt).to(device)
    t = {k: dev(a) for k, a in (("vx", vx), ("vy", vy), ("vz", vz))}
    t["x"] = dev(x) if x is not None else None
    return t
