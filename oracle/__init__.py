"""FP64 CPU oracle of the TRMC-R step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library:
the C source here is built on its own and loaded through ctypes.

The method follows Trazzi, Pareschi and Wennberg: Sec. 3 (time-relaxed
splitting and the Wild sum), Alg. 4.2 (split into collision sets), Alg. 4.3 and
4.4 (recursive collision trees, dummy collisions), Sec. 4.3 (adaptive depth),
Sec. 4.4 (tree-shape truncation, definitions def:2 and def:3, Alg. 4.6).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "trmc_oracle.c")
_LIB = os.path.join(_HERE, "libtrmc_oracle.so")

HOMOG, SLAB = 1, 2
NATURAL, FIXED, ADAPTIVE, ADAPTIVE_REUSE = 0, 1, 2, 3
WB_OFF, WB_MIN, WB_MEAN = 0, 1, 2
BC_SPECULAR, BC_INFLOW = 0, 1
MAJ_STEP, MAJ_LEVEL = 0, 1


def build() -> str:
    """Compile the oracle with gcc (contraction off, as the method's rounding conventions require)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fPIC", "-shared",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd, cwd=_HERE)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Desc(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint32), ("uid", ctypes.c_uint32),
        ("geometry", ctypes.c_uint32), ("n_cells", ctypes.c_uint32),
        ("length", ctypes.c_double), ("dt", ctypes.c_double), ("weight", ctypes.c_double),
        ("eps", ctypes.c_double), ("eps_cells", ctypes.POINTER(ctypes.c_double)),
        ("alpha", ctypes.c_double),
        ("trunc", ctypes.c_uint32), ("m_init", ctypes.c_uint32), ("m_cap", ctypes.c_uint32),
        ("delta1", ctypes.c_double), ("delta2", ctypes.c_double),
        ("wb", ctypes.c_uint32), ("wb_mmax", ctypes.c_uint32),
        ("bc", ctypes.c_uint32), ("in_left", ctypes.c_double * 3), ("in_right", ctypes.c_double * 3),
        ("majorant", ctypes.c_uint32),
    ]


class CellRecord(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint32), ("N0", ctypes.c_uint32), ("m_eff", ctypes.c_uint32),
        ("m_used", ctypes.c_uint32), ("attempts", ctypes.c_uint32), ("R0", ctypes.c_uint32),
        ("n_th", ctypes.c_uint32), ("borrowed", ctypes.c_uint32), ("folds", ctypes.c_uint32),
        ("m_state_after", ctypes.c_uint32), ("wb_th", ctypes.c_uint32),
        ("collisions", ctypes.c_uint64), ("dummies", ctypes.c_uint64),
        ("violations", ctypes.c_uint64), ("work_collisions", ctypes.c_uint64),
        ("q", ctypes.c_double), ("g", ctypes.c_double), ("E1", ctypes.c_double),
    ]


class AttemptRecord(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint32), ("N0", ctypes.c_uint32), ("m", ctypes.c_uint32), ("me", ctypes.c_uint32),
        ("mprev", ctypes.c_uint32), ("folds", ctypes.c_uint32),
        ("R0prev", ctypes.c_uint64), ("R0", ctypes.c_uint64), ("ncoll", ctypes.c_uint64),
        ("sum_R", ctypes.c_uint64), ("max_C", ctypes.c_uint64), ("coff_max", ctypes.c_uint64),
        ("borrowed", ctypes.c_uint64), ("n_th", ctypes.c_uint64),
    ]


class AttemptLog:
    """Integer outline of every attempt of the cell steps run on this thread
    inside the with-block (see orc_attempt): a list of dicts in .records."""

    def __init__(self, cap=1 << 16):
        self.buf = (AttemptRecord * cap)()
        self.cap = cap
        self.records = []

    def __enter__(self):
        lib().orc_attempt_log(self.buf, self.cap)
        return self

    def __exit__(self, *exc):
        k = lib().orc_attempt_log(None, 0)
        names = [f for f, _ in AttemptRecord._fields_]
        self.records = [{f: int(getattr(self.buf[i], f)) for f in names} for i in range(min(k, self.cap))]
        return False


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        u32, u64, dbl = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
        P = ctypes.POINTER
        L.orc_philox.argtypes = [P(u32), u32, u32, P(u32)]
        L.orc_philox.restype = None
        L.orc_exp_neg.argtypes = [dbl]
        L.orc_exp_neg.restype = dbl
        L.orc_grid_up.argtypes = [dbl]
        L.orc_grid_up.restype = dbl
        L.orc_perm.argtypes = [u32, u32, P(u32)]
        L.orc_perm.restype = u32
        L.orc_transport.argtypes = [P(dbl), P(dbl), dbl, dbl, u32]
        L.orc_transport.restype = u32
        L.orc_run.argtypes = [P(_Desc), P(u64), u64, P(dbl), P(dbl), P(dbl), P(dbl), P(u32), u32, u32,
                              P(CellRecord), P(u32)]
        L.orc_flux_inverse.argtypes = [dbl, dbl]
        L.orc_flux_inverse.restype = dbl
        L.orc_inflow_mean.argtypes = [dbl, dbl, dbl, dbl, dbl]
        L.orc_inflow_mean.restype = dbl
        L.orc_run.restype = ctypes.c_int
        L.orc_moments.argtypes = [u64, P(dbl), P(dbl), P(dbl), dbl, P(dbl)]
        L.orc_moments.restype = None
        L.orc_split.argtypes = [u32, u32, u32, u32, u32, dbl, u32, P(u64), P(u32)]
        L.orc_split.restype = ctypes.c_int
        L.orc_collide.argtypes = [P(dbl), P(dbl), dbl, dbl, dbl, dbl, dbl, P(dbl), P(dbl)]
        L.orc_collide.restype = ctypes.c_int
        L.orc_tree.argtypes = [u32, u32, u32, u32, u32, dbl, u32, u32, P(u64), P(u64), P(u64), P(u32),
                               P(u64), P(u64), u64, P(dbl), P(u32), P(u64)]
        L.orc_tree.restype = ctypes.c_int64
        L.orc_wb_len.argtypes = [dbl, dbl, u32]
        L.orc_wb_len.restype = dbl
        L.orc_attempt_log.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        L.orc_attempt_log.restype = ctypes.c_uint64
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def philox(ctr, key):
    """Philox4x32-10 block for counter ``ctr`` (4 words) and key ``key`` (2 words)."""
    c = np.asarray(ctr, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_p(c, ctypes.c_uint32), int(key[0]), int(key[1]), _p(out, ctypes.c_uint32))
    return out


def exp_neg(x: float) -> float:
    return lib().orc_exp_neg(float(x))


def grid_up(g: float) -> float:
    return lib().orc_grid_up(float(g))


def perm(i: int, n: int, keys) -> int:
    k = np.asarray(keys, dtype=np.uint32)
    return lib().orc_perm(int(i), int(n), _p(k, ctypes.c_uint32))


def transport(x: float, vx: float, dt: float, L: float, n_cells: int):
    xa = ctypes.c_double(x)
    va = ctypes.c_double(vx)
    c = lib().orc_transport(ctypes.byref(xa), ctypes.byref(va), dt, L, n_cells)
    return xa.value, va.value, c


def split(seed, uid, cell, step, n, q, m):
    """Collision-set sizes N_0..N_{m+1} (Alg. 4.2) and the effective depth."""
    N = np.zeros(m + 2, dtype=np.uint64)
    me = ctypes.c_uint32(0)
    lib().orc_split(seed, uid, cell, step, n, float(q), m, _p(N, ctypes.c_uint64), ctypes.byref(me))
    return N, me.value


def collide(a, b, xi1, xi2, xacc=0.0, alpha=0.0, g=1.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    oa = np.zeros(3)
    ob = np.zeros(3)
    acc = lib().orc_collide(_p(a, ctypes.c_double), _p(b, ctypes.c_double), xi1, xi2, xacc, alpha, g,
                            _p(oa, ctypes.c_double), _p(ob, ctypes.c_double))
    return oa, ob, bool(acc)


def flux_inverse(a: float, u: float) -> float:
    """Inward normal speed over sigma of a reservoir particle (reading R17) for the
    uniform u: the inverse of the flux-weighted half-range distribution."""
    return lib().orc_flux_inverse(float(a), float(u))


def inflow_mean(rho: float, u_in: float, T: float, weight: float, dt: float) -> float:
    """Expected particles entering through one end in one step."""
    return lib().orc_inflow_mean(float(rho), float(u_in), float(T), float(weight), float(dt))


def wb_len(a: float, b: float, kind: int) -> float:
    """Length of a collision's output from its inputs' lengths (Sec. 4.4)."""
    return lib().orc_wb_len(float(a), float(b), int(kind))


def tree(seed, uid, cell, step, n, q, m, kind=WB_OFF, cap=1 << 22):
    """Tree schedule of one cell (level order) and the lengths of its finals.

    Returns a dict: me, R0, R/C/first per level, j/rA/rB per collision and, for
    kind WB_MIN or WB_MEAN, finlen (finals listed level 1 first, by output rank)."""
    R = np.zeros(m + 2, dtype=np.uint64)
    C = np.zeros(m + 2, dtype=np.uint64)
    first = np.zeros(m + 2, dtype=np.uint64)
    j = np.zeros(cap, dtype=np.uint32)
    rA = np.zeros(cap, dtype=np.uint64)
    rB = np.zeros(cap, dtype=np.uint64)
    finlen = np.zeros(max(n, 1))
    me = ctypes.c_uint32(0)
    R0 = ctypes.c_uint64(0)
    nc = lib().orc_tree(seed, uid, cell, step, n, float(q), m, kind, _p(R, ctypes.c_uint64),
                        _p(C, ctypes.c_uint64), _p(first, ctypes.c_uint64), _p(j, ctypes.c_uint32),
                        _p(rA, ctypes.c_uint64), _p(rB, ctypes.c_uint64), cap, _p(finlen, ctypes.c_double),
                        ctypes.byref(me), ctypes.byref(R0))
    if nc < 0:
        raise ValueError("tree larger than cap")
    return {"me": me.value, "R0": R0.value, "R": R, "C": C, "first": first, "j": j[:nc], "rA": rA[:nc],
            "rB": rB[:nc], "finlen": finlen[:R0.value] if kind != WB_OFF else None}


@dataclass
class Instance:
    """State and parameters of one homogeneous solve or one 1-D slab."""
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    x: np.ndarray | None = None
    seed: int = 0
    uid: int = 0
    geometry: int = HOMOG
    n_cells: int = 1
    length: float = 1.0
    dt: float = 0.05
    weight: float | None = None
    eps: float = 1.0
    eps_cells: np.ndarray | None = None
    alpha: float = 0.0
    trunc: int = NATURAL
    m_init: int = 2
    m_cap: int = 64
    delta1: float = 0.005
    delta2: float = 0.01
    wb: int = WB_OFF
    wb_mmax: int = 5
    bc: int = BC_SPECULAR
    in_left: tuple | None = None   # reservoir (rho, u, T) at x = 0, u along +x
    in_right: tuple | None = None  # reservoir (rho, u, T) at x = length
    capacity: int | None = None    # open slab: room for entering particles
    majorant: int = MAJ_STEP       # MAJ_LEVEL: the VHS bound raised level by level (Remark 4.1)
    step: int = 0
    m_state: np.ndarray | None = None
    last: list | None = None

    def __post_init__(self):
        self.n_live = len(self.vx)
        cap = max(self.capacity or 0, self.n_live)

        def buf(a):
            b = np.zeros(cap)
            b[:self.n_live] = np.asarray(a, dtype=np.float64)
            return b
        self.vx, self.vy, self.vz = buf(self.vx), buf(self.vy), buf(self.vz)
        if self.x is not None:
            self.x = buf(self.x)
        if self.weight is None:
            self.weight = self.length / max(1, self.n_live)
        nc = self.n_cells if self.geometry == SLAB else 1
        if self.m_state is None:
            self.m_state = np.full(nc, self.m_init, dtype=np.uint32)
        if self.eps_cells is not None:
            self.eps_cells = np.ascontiguousarray(self.eps_cells, dtype=np.float64)

    @property
    def n(self) -> int:
        return self.n_live

    def _desc(self) -> _Desc:
        d = _Desc()
        d.seed, d.uid, d.geometry, d.n_cells = self.seed, self.uid, self.geometry, self.n_cells
        d.length, d.dt, d.weight, d.eps = self.length, self.dt, self.weight, self.eps
        d.eps_cells = _p(self.eps_cells, ctypes.c_double) if self.eps_cells is not None else None
        d.alpha = self.alpha
        d.trunc, d.m_init, d.m_cap = self.trunc, self.m_init, self.m_cap
        d.delta1, d.delta2 = self.delta1, self.delta2
        d.wb, d.wb_mmax = self.wb, self.wb_mmax
        d.bc = self.bc
        d.majorant = self.majorant
        if self.in_left is not None:
            d.in_left = (ctypes.c_double * 3)(*self.in_left)
        if self.in_right is not None:
            d.in_right = (ctypes.c_double * 3)(*self.in_right)
        return d

    def run(self, n_steps: int = 1):
        """Advance ``n_steps`` steps in place; keep the per-cell records of the last one."""
        nc = self.n_cells if self.geometry == SLAB else 1
        rec = (CellRecord * nc)()
        counts = np.zeros(nc, dtype=np.uint32)
        d = self._desc()
        xp = _p(self.x, ctypes.c_double) if self.x is not None else None
        n_io = ctypes.c_uint64(self.n_live)
        rc = lib().orc_run(ctypes.byref(d), ctypes.byref(n_io), len(self.vx), xp, _p(self.vx, ctypes.c_double),
                           _p(self.vy, ctypes.c_double), _p(self.vz, ctypes.c_double),
                           _p(self.m_state, ctypes.c_uint32), self.step, n_steps, rec,
                           _p(counts, ctypes.c_uint32))
        if rc != 0:
            raise RuntimeError(f"oracle run failed ({rc})")
        self.n_live = int(n_io.value)
        self.step += n_steps
        self.last = [rec[i] for i in range(nc)]
        self.counts = counts
        return self.last

    def moments(self):
        """Per-cell moments [rho, ux, uy, uz, T, Pxx, Pyy, Pzz, M4] of the current state."""
        nc = self.n_cells if self.geometry == SLAB else 1
        vol = self.length / nc if self.geometry == SLAB else self.length
        out = np.zeros((nc, 9))
        if self.geometry == SLAB:
            starts = (np.concatenate([[0], np.cumsum(self.counts.astype(np.int64))]).astype(np.int64)
                      if hasattr(self, "counts") else None)
            if starts is None:
                raise RuntimeError("moments of a slab need at least one step (cells are sorted by it)")
        else:
            starts = np.array([0, self.n])
        for c in range(nc):
            a, b = int(starts[c]), int(starts[c + 1])
            vx, vy, vz = self.vx[a:b], self.vy[a:b], self.vz[a:b]
            o = np.zeros(9)
            lib().orc_moments(b - a, _p(np.ascontiguousarray(vx), ctypes.c_double),
                              _p(np.ascontiguousarray(vy), ctypes.c_double),
                              _p(np.ascontiguousarray(vz), ctypes.c_double), self.weight / vol,
                              _p(o, ctypes.c_double))
            out[c] = o
        return out
