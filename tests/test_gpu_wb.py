"""GPU parity of the tree-shape truncation (TRMC-WB, Sec. 4.4) against the oracle.

FP64: integers exact (including the count of finals thermalized by tree shape),
velocities within the parity tolerance, for both length definitions (def:2 and
def:3), Maxwell molecules and hard spheres, fixed and natural truncation, a
homogeneous cell spanning several 512-particle tiles with a ragged tail, and a
slab.  FP32: momentum and energy kept at every step.  An instance with
tree-shape truncation stepped beside a plain one gives the result it gives alone.
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


@pytest.fixture(scope="module")
def trmc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible ROCm GPU"
    import paper_1009_2768_amd as T
    T.load()
    return T


def say(*a):
    print("[gpu-case]", *a, flush=True)


def _homog(T, n, wb, mmax, alpha, eps, trunc, m, precision, uid, init="bimax"):
    if init == "bkw":
        vx, vy, vz = W.bkw(n, 0.6, seed=5, stream=uid)
    else:
        vx, vy, vz = W.bimaxwellian(n, seed=5, stream=uid)
    inst = T.Instance(n_particles=n, eps=eps, alpha=alpha, trunc=trunc, m_init=m, m_cap=64, uid=uid, seed=5,
                      precision=precision, wb=wb, wb_mmax=mmax)
    return inst, {"vx": vx, "vy": vy, "vz": vz}


def _run(T, insts, arrays, steps):
    parts = [T.device_particles(a["vx"], a["vy"], a["vz"], a.get("x"), i.precision) for i, a in zip(insts, arrays)]
    ctx = T.Context(insts, parts)
    ctx.step(steps)
    out = [(ctx.read(k), ctx.moments(k)) for k in range(len(insts))]
    ctx.close()
    return out


CASES = [
    # (n, wb, mmax, alpha, eps, trunc, m)
    (3000, 1, 2, 0.0, 0.02, 1, 16),
    (3000, 2, 2, 0.0, 0.02, 1, 16),
    (6100, 2, 3, 1.0, 0.1, 1, 16),
    (6100, 1, 2, 1.0, 0.2, 1, 24),
    (2500, 2, 4, 0.0, 0.01, 0, 64),   # natural truncation, deep trees
    (700, 1, 1, 0.0, 0.05, 1, 8),     # m_max = 1: every final whose inputs are both collision outputs
]


@pytest.mark.parametrize("case", CASES)
def test_homogeneous_fp64_matches_oracle(trmc, orc, case):
    T = trmc
    n, wb, mmax, alpha, eps, trunc, m = case
    inst, a = _homog(T, n, wb, mmax, alpha, eps, trunc, m, T.FP64, uid=40 + CASES.index(case))
    say(f"wb fp64 n={n} def={wb} mmax={mmax} alpha={alpha} eps={eps} trunc={trunc} m={m}")
    (got, mom), = _run(T, [inst], [a], 3)
    o = oracle_of(orc, inst, a)
    o.run(3)
    assert int(mom["wb_thermalized"][0]) > 0
    compare(o, got, mom, 1)


def test_slab_fp64_matches_oracle(trmc, orc):
    T = trmc
    nc = 40
    x, vx, vy, vz, w = W.sod(nc, 300, 40, seed=8)
    inst = T.Instance(n_particles=len(x), geometry=T.SLAB1D, n_cells=nc, dt=W.sod_dt(1.0, nc), eps=0.005,
                      alpha=1.0, trunc=T.FIXED, m_init=12, m_cap=64, particle_weight=w, uid=51, seed=8,
                      precision=T.FP64, wb=T.WB_MEAN, wb_mmax=2)
    a = {"x": x, "vx": vx, "vy": vy, "vz": vz}
    say(f"wb slab fp64: {nc} cells, {len(x)} particles")
    (got, mom), = _run(T, [inst], [a], 3)
    o = oracle_of(orc, inst, a)
    o.run(3)
    assert int(mom["wb_thermalized"].sum()) > 0
    compare(o, got, mom, nc)


def test_fp32_conserves_every_step(trmc):
    T = trmc
    inst, a = _homog(T, 20000, T.WB_MIN, 2, 1.0, 0.2, T.FIXED, 24, T.FP32_MIXED, uid=52)
    say("wb fp32 conservation, n=20000")
    parts = [T.device_particles(a["vx"], a["vy"], a["vz"], None, T.FP32_MIXED)]
    ctx = T.Context([inst], parts)

    def sums(g):
        v = np.stack([g["vx"], g["vy"], g["vz"]]).astype(np.float64)
        return v.sum(1), np.abs(v).sum(), float((v * v).sum())

    p0, s0, e0 = sums(ctx.read(0))
    th = 0
    for _ in range(4):
        ctx.step(1)
        p1, s1, e1 = sums(ctx.read(0))
        th += int(ctx.moments(0)["wb_thermalized"][0])
        assert np.abs(p1 - p0).max() <= 1e-6 * s0
        assert abs(e1 - e0) <= 1e-6 * e0
        p0, s0, e0 = p1, s1, e1
    ctx.close()
    assert th > 0


def test_beside_a_plain_instance_equals_alone(trmc):
    T = trmc
    a_inst, a = _homog(T, 5000, T.WB_MEAN, 2, 0.0, 0.02, T.FIXED, 16, T.FP64, uid=53)
    b_inst, b = _homog(T, 5000, T.WB_OFF, 5, 0.0, 0.02, T.ADAPTIVE, 2, T.FP64, uid=54, init="bkw")
    say("wb instance beside a plain one")
    (ga, ma), (gb, mb) = _run(T, [a_inst, b_inst], [a, b], 3)
    (ga1, ma1), = _run(T, [a_inst], [a], 3)
    (gb1, mb1), = _run(T, [b_inst], [b], 3)
    for k in ("vx", "vy", "vz"):
        np.testing.assert_array_equal(ga[k], ga1[k])
        np.testing.assert_array_equal(gb[k], gb1[k])
    assert int(ma["wb_thermalized"][0]) == int(ma1["wb_thermalized"][0]) > 0
    assert int(mb["wb_thermalized"][0]) == 0
