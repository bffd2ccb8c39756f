"""GPU parity of the adaptive depth that keeps rejected attempts (Sec. 4.3,
collisions of the wrong depth reused) against the oracle.

FP64: integers exact (attempts, collisions, leaves, thermalized, depths) and
velocities within the parity tolerance, with rejections forced down to m_cap
and with the paper's thresholds over several steps, Maxwell molecules and hard
spheres, cells from a few hundred particles to several tiles with a ragged tail,
and a slab.  FP32: momentum and energy kept at every step.  Beside a plain
adaptive instance, each gives the result it gives alone.
"""
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from test_gpu_parity import compare, oracle_of  # noqa: E402

FORCE = dict(delta1=1e-12, delta2=2e-12)


@pytest.fixture(scope="module")
def trmc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible ROCm GPU"
    import paper_1009_2768_amd as T
    T.load()
    return T


def say(*a):
    print("[gpu-case]", *a, flush=True)


def _run(T, insts, arrays, steps):
    parts = [T.device_particles(a["vx"], a["vy"], a["vz"], a.get("x"), i.precision) for i, a in zip(insts, arrays)]
    ctx = T.Context(insts, parts)
    ctx.step(steps)
    out = [(ctx.read(k), ctx.moments(k)) for k in range(len(insts))]
    ctx.close()
    return out


CASES = [
    # (n, alpha, eps, m_init, m_cap, forced, steps, init)
    (3000, 0.0, 0.05, 2, 16, True, 1, "bkw"),
    (6100, 1.0, 0.3, 2, 64, True, 1, "bimax"),
    (700, 0.0, 0.02, 2, 8, True, 2, "bkw"),
    (20000, 1.0, 0.5, 2, 64, False, 4, "bimax"),
    (5000, 0.0, 0.1, 2, 64, False, 4, "bkw"),
    (300, 1.0, 0.05, 4, 32, True, 2, "bimax"),
]


@pytest.mark.parametrize("case", CASES)
def test_homogeneous_fp64_matches_oracle(trmc, orc, case):
    T = trmc
    n, alpha, eps, m0, mcap, forced, steps, init = case
    uid = 60 + CASES.index(case)
    a = W.bkw(n, 0.6, seed=6, stream=uid) if init == "bkw" else W.bimaxwellian(n, seed=6, stream=uid)
    arr = {"vx": a[0], "vy": a[1], "vz": a[2]}
    kw = FORCE if forced else {}
    inst = T.Instance(n_particles=n, eps=eps, alpha=alpha, trunc=T.ADAPTIVE_REUSE, m_init=m0, m_cap=mcap, uid=uid,
                      seed=6, precision=T.FP64, **kw)
    say(f"reuse fp64 n={n} alpha={alpha} eps={eps} m={m0}..{mcap} forced={forced} steps={steps}")
    (got, mom), = _run(T, [inst], [arr], steps)
    o = oracle_of(orc, inst, arr)
    o.run(steps)
    if forced and steps == 1:
        assert int(mom["attempts"][0]) > 1  # the step really extended rejected attempts
    compare(o, got, mom, 1)
    assert int(mom["work_collisions"][0]) == int(mom["collisions"][0])


def test_slab_fp64_matches_oracle(trmc, orc):
    T = trmc
    nc = 40
    x, vx, vy, vz, w = W.sod(nc, 300, 40, seed=9)
    inst = T.Instance(n_particles=len(x), geometry=T.SLAB1D, n_cells=nc, dt=W.sod_dt(1.0, nc), eps=0.01,
                      alpha=1.0, trunc=T.ADAPTIVE_REUSE, m_init=2, m_cap=64, particle_weight=w, uid=71, seed=9,
                      precision=T.FP64)
    a = {"x": x, "vx": vx, "vy": vy, "vz": vz}
    say(f"reuse slab fp64: {nc} cells, {len(x)} particles, 4 steps")
    (got, mom), = _run(T, [inst], [a], 4)
    o = oracle_of(orc, inst, a)
    o.run(4)
    compare(o, got, mom, nc)


def test_fp32_conserves_every_step(trmc):
    T = trmc
    a = W.bimaxwellian(20000, seed=6, stream=72)
    inst = T.Instance(n_particles=20000, eps=0.3, alpha=1.0, trunc=T.ADAPTIVE_REUSE, m_init=2, m_cap=64, uid=72,
                      seed=6, precision=T.FP32_MIXED)
    say("reuse fp32 conservation, n=20000")
    ctx = T.Context([inst], [T.device_particles(a[0], a[1], a[2], None, T.FP32_MIXED)])

    def sums(g):
        v = np.stack([g["vx"], g["vy"], g["vz"]]).astype(np.float64)
        return v.sum(1), np.abs(v).sum(), float((v * v).sum())

    p0, s0, e0 = sums(ctx.read(0))
    for _ in range(4):
        ctx.step(1)
        p1, s1, e1 = sums(ctx.read(0))
        assert np.abs(p1 - p0).max() <= 1e-6 * s0
        assert abs(e1 - e0) <= 1e-6 * e0
        p0, s0, e0 = p1, s1, e1
    ctx.close()


def test_beside_plain_adaptive_equals_alone(trmc):
    T = trmc
    a = W.bkw(5000, 0.6, seed=6, stream=73)
    b = W.bkw(5000, 0.6, seed=6, stream=74)
    A = T.Instance(n_particles=5000, eps=0.05, trunc=T.ADAPTIVE_REUSE, m_init=2, m_cap=64, uid=73, seed=6,
                   precision=T.FP64)
    B = T.Instance(n_particles=5000, eps=0.05, trunc=T.ADAPTIVE, m_init=2, m_cap=64, uid=74, seed=6,
                   precision=T.FP64)
    aa = {"vx": a[0], "vy": a[1], "vz": a[2]}
    bb = {"vx": b[0], "vy": b[1], "vz": b[2]}
    say("reuse instance beside a plain adaptive one")
    (ga, ma), (gb, mb) = _run(T, [A, B], [aa, bb], 3)
    (ga1, _), = _run(T, [A], [aa], 3)
    (gb1, _), = _run(T, [B], [bb], 3)
    for k in ("vx", "vy", "vz"):
        np.testing.assert_array_equal(ga[k], ga1[k])
        np.testing.assert_array_equal(gb[k], gb1[k])


def test_wave_path_matches_oracle(trmc, orc):
    """Small cells on the wave-per-cell path (eight cells per workgroup)."""
    T = trmc
    sizes = [256, 300, 511, 700, 1000, 1500, 1999, 450, 820]
    insts, arrs = [], []
    for k, n in enumerate(sizes):
        a = W.bkw(n, 0.6, seed=7, stream=80 + k) if k % 2 else W.bimaxwellian(n, seed=7, stream=80 + k)
        arrs.append({"vx": a[0], "vy": a[1], "vz": a[2]})
        kw = FORCE if k % 3 == 0 else {}
        insts.append(T.Instance(n_particles=n, eps=[0.02, 0.1, 0.5][k % 3], alpha=float(k % 2),
                                trunc=T.ADAPTIVE_REUSE, m_init=2, m_cap=64, uid=80 + k, seed=7, precision=T.FP64,
                                **kw))
    say(f"reuse fp64 wave path: {len(sizes)} cells of {min(sizes)}..{max(sizes)} particles, 3 steps")
    parts = [T.device_particles(a["vx"], a["vy"], a["vz"], None, T.FP64) for a in arrs]
    ctx = T.Context(insts, parts)
    table = [0] * T.SCHED_BUCKETS
    for b in range(8, 11):
        table[b] = T.PATH_WAVE
    ctx.set_schedule(table)
    ctx.step(3)
    res = [(ctx.read(k), ctx.moments(k)) for k in range(len(insts))]
    ctx.close()
    redone = 0
    for inst, a, (got, mom) in zip(insts, arrs, res):
        o = oracle_of(orc, inst, a)
        o.run(3)
        compare(o, got, mom, 1)
        redone += int(mom["attempts"][0] > 1)
    assert redone > 0
