"""GPU: FP32-mixed path against the FP64 oracle, batching and serving determinism.

FP32-mixed keeps velocities and collision arithmetic in float and the cell sums
and the conservation rescale in double.  With Maxwell molecules and a fixed depth
the integer schedule equals the FP64 oracle's (same draws, q does not depend on
the velocities), so the FP32 trajectory is a rounding perturbation of the oracle's;
otherwise FP32 is checked by conservation (<= 1e-6 relative) and by cell moments
within 3 sigma of an oracle ensemble.  Serving: each result is the same alone
and in the mix (bitwise).
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


def inst_arrays(T, n, eps, alpha, trunc, prec, init="bimax", uid=0, m_init=2, stream=0, dt=0.05):
    vx, vy, vz = W.bimaxwellian(n, stream=stream) if init == "bimax" else W.bkw(n, 0.6, stream=stream)
    inst = T.Instance(n_particles=n, eps=eps, alpha=alpha, trunc=trunc, m_init=m_init, m_cap=64, uid=uid,
                      precision=prec, dt=dt)
    return inst, {"vx": vx, "vy": vy, "vz": vz}


def run(T, insts, arrays, steps):
    parts = [T.device_particles(a["vx"], a["vy"], a["vz"], a.get("x"), i.precision) for i, a in zip(insts, arrays)]
    ctx = T.Context(insts, parts)
    ctx.step(steps)
    out = [(ctx.read(k), ctx.moments(k)) for k in range(len(insts))]
    ctx.close()
    return out


def test_fp32_maxwell_fixed_depth_tracks_fp64_oracle(trmc, orc):
    say("fp32 maxwell fixed depth vs fp64 oracle")
    inst, a = inst_arrays(trmc, 10000, 0.3, 0.0, trmc.FIXED, trmc.FP32_MIXED, init="bkw", m_init=3)
    (got, mom), = run(trmc, [inst], [a], 3)
    a32 = {k: v.astype(np.float32).astype(np.float64) for k, v in a.items()}
    o = orc.Instance(a32["vx"], a32["vy"], a32["vz"], eps=0.3, dt=0.05, trunc=orc.FIXED, m_init=3, m_cap=64,
                     weight=1.0 / 10000)
    o.run(3)
    r = o.last[0]
    for gk, ok in (("N0", "N0"), ("R0", "R0"), ("thermalized", "n_th"), ("collisions", "collisions"),
                   ("m_eff", "m_eff")):
        assert int(mom[gk][0]) == int(getattr(r, ok)), gk
    T_cell = (o.vx.var() + o.vy.var() + o.vz.var()) / 3
    err = max(float(np.abs(got[k].astype(np.float64) - getattr(o, k)).max()) for k in ("vx", "vy", "vz"))
    err /= math.sqrt(T_cell)
    say(f"fp32 vs fp64 oracle: max |dv|/sqrt(T) = {err:.2e}")
    assert err < 1e-5


@pytest.mark.parametrize("alpha,eps", [(1.0, 0.05), (0.0, 0.2), (1.0, 1e-3)])
def test_fp32_conservation(trmc, alpha, eps):
    say("fp32 conservation", alpha, eps)
    inst, a = inst_arrays(trmc, 20000, eps, alpha, trmc.ADAPTIVE, trmc.FP32_MIXED, uid=3)
    parts = [trmc.device_particles(a["vx"], a["vy"], a["vz"], None, inst.precision)]
    ctx = trmc.Context([inst], parts)
    prev = ctx.read(0)
    for _ in range(5):
        ctx.step(1)
        cur = ctx.read(0)
        v0 = np.stack([prev["vx"], prev["vy"], prev["vz"]], 1).astype(np.float64)
        v1 = np.stack([cur["vx"], cur["vy"], cur["vz"]], 1).astype(np.float64)
        dp = np.abs(v1.sum(0) - v0.sum(0)).max() / np.abs(v0).sum()
        de = abs((v1**2).sum() - (v0**2).sum()) / (v0**2).sum()
        assert dp <= 1e-6 and de <= 1e-6, (dp, de)
        prev = cur
    ctx.close()


@pytest.mark.parametrize("n,eps,alpha", [(1_000_000, 1e-4, 1.0), (262_144, 0.05 / math.log(2.0 * 262_144), 0.0)])
def test_fp32_conservation_on_the_tile_path(trmc, n, eps, alpha):
    """FP32 conservation at every step on the tile path at the serving stream's
    large sizes, where cells predicted wholly thermalized take the whole cell's
    sums from the tile sums (and, at the threshold eps, predictions fail)."""
    say("fp32 conservation, tile path", n, eps, alpha)
    inst, a = inst_arrays(trmc, n, eps, alpha, trmc.ADAPTIVE, trmc.FP32_MIXED, uid=43)
    parts = [trmc.device_particles(a["vx"], a["vy"], a["vz"], None, inst.precision)]
    ctx = trmc.Context([inst], parts)
    ctx.set_schedule([trmc.PATH_TILED] * trmc.SCHED_BUCKETS)
    prev = ctx.read(0)
    for _ in range(6):
        ctx.step(1)
        cur = ctx.read(0)
        v0 = np.stack([prev["vx"], prev["vy"], prev["vz"]], 1).astype(np.float64)
        v1 = np.stack([cur["vx"], cur["vy"], cur["vz"]], 1).astype(np.float64)
        dp = np.abs(v1.sum(0) - v0.sum(0)).max() / np.abs(v0).sum()
        de = abs((v1**2).sum() - (v0**2).sum()) / (v0**2).sum()
        assert dp <= 1e-6 and de <= 1e-6, (dp, de)
        prev = cur
    ctx.close()


def test_fp32_moments_within_3_sigma_of_oracle_ensemble(trmc, orc):
    """Hard spheres, adaptive depth: per-moment ensemble means (24 replicas) of the
    FP32 path within 3 sigma of the FP64 oracle's."""
    say("fp32 moments vs oracle ensemble")
    R, n, steps = 24, 4000, 3
    insts, arrays = [], []
    for r in range(R):
        inst, a = inst_arrays(trmc, n, 0.05, 1.0, trmc.ADAPTIVE, trmc.FP32_MIXED, uid=r, stream=r)
        insts.append(inst)
        arrays.append(a)
    res = run(trmc, insts, arrays, steps)
    keys = ["T", "Pxx", "Pyy", "M4"]
    g = np.array([[m[k][0] for k in keys] for _, m in res])
    o = []
    for r in range(R):
        oi = orc.Instance(arrays[r]["vx"], arrays[r]["vy"], arrays[r]["vz"], eps=0.05, dt=0.05, alpha=1.0,
                          trunc=orc.ADAPTIVE, m_init=2, m_cap=64, uid=r, weight=1.0 / n)
        oi.run(steps)
        m = oi.moments()[0]
        o.append([m[4], m[5], m[6], m[8]])
    o = np.array(o)
    se = np.sqrt(g.var(0, ddof=1) / R + o.var(0, ddof=1) / R)
    z = np.abs(g.mean(0) - o.mean(0)) / se
    say("fp32 vs fp64 ensemble z-scores", dict(zip(keys, np.round(z, 3))))
    assert np.all(z < 3.0), z


def test_fp32_slab_counts_and_conservation(trmc, orc):
    say("fp32 slab")
    x, vx, vy, vz, w = W.sod(40, 200, 25, seed=5)
    kw = dict(n_particles=len(x), geometry=trmc.SLAB1D, n_cells=40, dt=W.sod_dt(1.0, 40), eps=0.01, alpha=1.0,
              trunc=trmc.ADAPTIVE, particle_weight=w, uid=9)
    inst = trmc.Instance(precision=trmc.FP32_MIXED, **kw)
    (got, mom), = run(trmc, [inst], [{"x": x, "vx": vx, "vy": vy, "vz": vz}], 6)
    assert int(mom["n"].sum()) == len(x)
    e0 = (vx.astype(np.float32).astype(np.float64) ** 2 + vy.astype(np.float32).astype(np.float64) ** 2
          + vz.astype(np.float32).astype(np.float64) ** 2).sum()
    e1 = (got["vx"].astype(np.float64) ** 2 + got["vy"].astype(np.float64) ** 2
          + got["vz"].astype(np.float64) ** 2).sum()
    assert abs(e1 - e0) / e0 <= 1e-6
    assert np.all((got["x"] >= 0) & (got["x"] <= 1))
    o = orc.Instance(vx, vy, vz, x=x, geometry=orc.SLAB, n_cells=40, dt=W.sod_dt(1.0, 40), eps=0.01, alpha=1.0,
                     trunc=orc.ADAPTIVE, weight=w, uid=9)
    o.run(6)
    # float transport may move a particle across a cell face differently: counts agree closely
    assert np.abs(mom["n"].astype(int) - o.counts.astype(int)).sum() <= 0.01 * len(x)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_alone_equals_in_mix(trmc, prec):
    say("alone vs mix", prec)
    P = trmc.FP64 if prec == "fp64" else trmc.FP32_MIXED
    target, ta = inst_arrays(trmc, 3000, 0.05, 1.0, trmc.ADAPTIVE, P, uid=77, stream=77)
    (alone, _), = run(trmc, [target], [ta], 4)
    others, oa = [], []
    for k in range(6):
        i, a = inst_arrays(trmc, 500 + 700 * k, 0.01 * (k + 1), float(k % 2), trmc.ADAPTIVE, P, uid=k, stream=k)
        others.append(i)
        oa.append(a)
    res = run(trmc, others[:3] + [target] + others[3:], oa[:3] + [ta] + oa[3:], 4)
    mixed = res[3][0]
    for k in ("vx", "vy", "vz"):
        assert np.array_equal(alone[k], mixed[k])


def test_admission_while_running(trmc):
    """Serving: an instance admitted after others have run gives the same result
    as alone; retiring an instance does not disturb the others."""
    say("admit while running")
    P = trmc.FP32_MIXED
    a_inst, a_arr = inst_arrays(trmc, 5000, 0.05, 1.0, trmc.ADAPTIVE, P, uid=1, stream=1)
    b_inst, b_arr = inst_arrays(trmc, 3000, 0.2, 0.0, trmc.ADAPTIVE, P, uid=2, stream=2)
    c_inst, c_arr = inst_arrays(trmc, 2000, 0.01, 1.0, trmc.ADAPTIVE, P, uid=3, stream=3)
    (a_alone, _), = run(trmc, [a_inst], [a_arr], 5)
    (b_alone, _), = run(trmc, [b_inst], [b_arr], 3)
    ctx = trmc.Context([a_inst, c_inst],
                       [trmc.device_particles(a_arr["vx"], a_arr["vy"], a_arr["vz"], None, P),
                        trmc.device_particles(c_arr["vx"], c_arr["vy"], c_arr["vz"], None, P)],
                       max_instances=4, max_cells=8)
    ctx.step(2)
    ctx.retire(1)
    sb = ctx.admit(b_inst, trmc.device_particles(b_arr["vx"], b_arr["vy"], b_arr["vz"], None, P))
    ctx.step(3)
    got_a = ctx.read(0)
    got_b = ctx.read(sb)
    ctx.close()
    for k in ("vx", "vy", "vz"):
        assert np.array_equal(a_alone[k], got_a[k])
        assert np.array_equal(b_alone[k], got_b[k])


def test_restart_bitwise(trmc):
    say("restart")
    x, vx, vy, vz, w = W.sod(16, 100, 12, seed=2)
    kw = dict(n_particles=len(x), geometry=trmc.SLAB1D, n_cells=16, dt=W.sod_dt(1.0, 16), eps=0.02, alpha=1.0,
              trunc=trmc.ADAPTIVE, particle_weight=w, uid=4, precision=trmc.FP64)
    full = trmc.Instance(**kw)
    (ref, _), = run(trmc, [full], [{"x": x, "vx": vx, "vy": vy, "vz": vz}], 8)
    half = trmc.Instance(**kw)
    parts = [trmc.device_particles(vx, vy, vz, x, trmc.FP64)]
    ctx = trmc.Context([half], parts)
    ctx.step(4)
    mid = ctx.read(0)
    ctx.close()
    assert mid["step"] == 4
    again = trmc.Instance(step0=4, m_state0=mid["m_state"], **kw)
    (out, _), = run(trmc, [again], [mid], 4)
    for k in ("x", "vx", "vy", "vz"):
        assert np.array_equal(ref[k], out[k]), k
