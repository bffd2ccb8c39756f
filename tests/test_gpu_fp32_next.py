"""GPU: the FP32-mixed path of the tree-shape truncation, the adaptive depth that
keeps rejected attempts and the open slab, against the FP64 oracle.

* Tree-shape truncation, Maxwell molecules, fixed depth, definition def:2 (integer
  lengths): the integer schedule equals the oracle's, so every counter is exact,
  and every particle that is not thermalized tracks the oracle to 1e-5 of the
  thermal speed.  Thermalized particles take FP32 Box-Muller normals from 24-bit
  uniforms, which differ from the oracle's FP64 normals by up to a few 1e-3 in the
  tails; they are checked through the cell's moments (1e-4 relative).
* Adaptive depth with reuse, hard spheres: per-moment ensemble means (24 replicas)
  within 3 sigma of the oracle's.
* Open slab: the particle count after 20 steps, over 12 replicas, within 3 sigma
  of the oracle's; per-step conservation does not apply (the ends are open).
"""
import math
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trmc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible ROCm GPU"
    import paper_1009_2768_amd as T
    T.load()
    return T


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _run(T, insts, arrays, steps, capacity=None):
    parts = [T.device_particles(a["vx"], a["vy"], a["vz"], a.get("x"), i.precision,
                                capacity=i.n_particles if i.bc else None) for i, a in zip(insts, arrays)]
    ctx = T.Context(insts, parts)
    ctx.step(steps)
    out = [(ctx.read(k), ctx.moments(k), ctx.count(k)) for k in range(len(insts))]
    ctx.close()
    return out


def test_fp32_tree_shape_truncation_tracks_fp64_oracle(trmc, orc):
    T = trmc
    n = 10000
    vx, vy, vz = W.bkw(n, 0.6, seed=4, stream=5)
    inst = T.Instance(n_particles=n, eps=0.02, alpha=0.0, trunc=T.FIXED, m_init=12, m_cap=64, uid=101, seed=4,
                      precision=T.FP32_MIXED, wb=T.WB_MIN, wb_mmax=2)
    say("fp32 tree-shape truncation (def:2) vs fp64 oracle")
    (got, mom, _), = _run(T, [inst], [{"vx": vx, "vy": vy, "vz": vz}], 3)
    a32 = [np.asarray(v, dtype=np.float32).astype(np.float64) for v in (vx, vy, vz)]
    o = orc.Instance(*a32, eps=0.02, dt=0.05, trunc=orc.FIXED, m_init=12, m_cap=64, weight=1.0 / n, uid=101, seed=4,
                     wb=orc.WB_MIN, wb_mmax=2)
    o.run(3)
    r = o.last[0]
    for gk, ok in (("N0", "N0"), ("R0", "R0"), ("thermalized", "n_th"), ("wb_thermalized", "wb_th"),
                   ("collisions", "collisions"), ("m_eff", "m_eff")):
        assert int(mom[gk][0]) == int(getattr(r, ok)), gk
    assert int(mom["wb_thermalized"][0]) > 0
    T_cell = (o.vx[:n].var() + o.vy[:n].var() + o.vz[:n].var()) / 3
    d = np.max([np.abs(got[k].astype(np.float64) - getattr(o, k)[:n]) for k in ("vx", "vy", "vz")], 0)
    d /= math.sqrt(T_cell)
    off = int((d > 1e-5).sum())
    say(f"  {off} of {n} particles beyond 1e-5 (thermalized {r.n_th}); max |dv|/sqrt(T) = {d.max():.2e}")
    assert off <= r.n_th
    assert d.max() < 2e-2
    g = np.stack([got["vx"], got["vy"], got["vz"]]).astype(np.float64)
    ov = np.stack([o.vx[:n], o.vy[:n], o.vz[:n]])
    for f in (lambda v: v.var(1), lambda v: ((v * v).sum(0) ** 2).mean()):
        assert np.allclose(f(g), f(ov), rtol=1e-4)


def test_fp32_reuse_moments_within_3_sigma_of_oracle_ensemble(trmc, orc):
    T = trmc
    R, n, steps = 24, 4000, 3
    insts, arrays = [], []
    for r in range(R):
        a = W.bimaxwellian(n, seed=0, stream=300 + r)
        insts.append(T.Instance(n_particles=n, eps=0.05, alpha=1.0, trunc=T.ADAPTIVE_REUSE, m_init=2, m_cap=64,
                                uid=300 + r, precision=T.FP32_MIXED))
        arrays.append({"vx": a[0], "vy": a[1], "vz": a[2]})
    say("fp32 reuse moments vs oracle ensemble")
    res = _run(T, insts, arrays, steps)
    keys = ["T", "Pxx", "Pyy", "M4"]
    g = np.array([[m[k][0] for k in keys] for _, m, _ in res])
    o = []
    for r in range(R):
        oi = orc.Instance(arrays[r]["vx"], arrays[r]["vy"], arrays[r]["vz"], eps=0.05, dt=0.05, alpha=1.0,
                          trunc=orc.ADAPTIVE_REUSE, m_init=2, m_cap=64, uid=300 + r, weight=1.0 / n)
        oi.run(steps)
        m = oi.moments()[0]
        o.append([m[4], m[5], m[6], m[8]])
    o = np.array(o)
    se = np.sqrt(g.var(0, ddof=1) / R + o.var(0, ddof=1) / R)
    z = np.abs(g.mean(0) - o.mean(0)) / se
    say("  z-scores", dict(zip(keys, np.round(z, 3))))
    assert np.all(z < 3.0), z


def test_fp32_open_slab_count_within_3_sigma_of_oracle(trmc, orc):
    T = trmc
    R, nc, steps = 12, 20, 20
    insts, arrays, o_counts = [], [], []
    for r in range(R):
        x, vx, vy, vz, w, up, down, cap = W.shock(nc, 60, seed=9, stream=r)
        kw = dict(geometry=T.SLAB1D, n_cells=nc, length=1.0, dt=W.shock_dt(1.0, nc), eps=0.1, alpha=1.0,
                  trunc=T.ADAPTIVE, m_init=2, m_cap=64, particle_weight=w, uid=400 + r, seed=9)
        insts.append(T.Instance(n_particles=cap, precision=T.FP32_MIXED, bc=T.BC_INFLOW, n_live0=len(x),
                                in_left=up, in_right=down, **kw))
        arrays.append({"x": x, "vx": vx, "vy": vy, "vz": vz})
        oi = orc.Instance(vx, vy, vz, x=x, geometry=orc.SLAB, n_cells=nc, length=1.0, dt=kw["dt"], eps=0.1,
                          alpha=1.0, trunc=orc.ADAPTIVE, m_init=2, m_cap=64, weight=w, uid=400 + r, seed=9,
                          bc=orc.BC_INFLOW, in_left=up, in_right=down, capacity=cap)
        oi.run(steps)
        o_counts.append(oi.n)
    say("fp32 open slab counts vs oracle")
    res = _run(T, insts, arrays, steps)
    g = np.array([c for _, _, c in res], dtype=np.float64)
    o = np.array(o_counts, dtype=np.float64)
    se = math.sqrt(g.var(ddof=1) / R + o.var(ddof=1) / R)
    z = abs(g.mean() - o.mean()) / se
    say(f"  mean count gpu {g.mean():.1f} oracle {o.mean():.1f}, z {z:.2f}")
    assert z < 3.0
