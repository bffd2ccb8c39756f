"""Pins of the adaptive depth with reuse of a rejected attempt's collisions
(Sec. 4.3: the collisions computed at depth m are kept, the Maxwellian part
(1 - tau)^(m+1) M is dropped, the levels m+1..2m are added by the recursive
collision process and the new remainder is sampled from the Maxwellian).

* An attempt accepted at once is the plain adaptive step, bit for bit.
* With rejections forced (delta2 below any E_1), the accepted step has the
  relaxation law of the Wild sum truncated at the final depth (the closed forms
  of the stress and M4 decay for Maxwell molecules), not that of the first depth.
* No work is discarded: the work counter equals the collisions of the result.
* Momentum and energy are kept.
"""
import math

import numpy as np
import pytest

import workloads as W
from test_oracle_physics import _tau, r2, r4

FORCE = dict(delta1=1e-12, delta2=2e-12)  # every E_1 > delta2: redo until m_cap


def test_accepted_at_once_equals_plain_adaptive(orc):
    vx, vy, vz = W.bimaxwellian(5000, seed=3)
    kw = dict(eps=5.0, dt=0.05, alpha=1.0, m_init=4, m_cap=64)
    a = orc.Instance(vx, vy, vz, trunc=orc.ADAPTIVE, **kw)
    b = orc.Instance(vx, vy, vz, trunc=orc.ADAPTIVE_REUSE, **kw)
    for _ in range(4):
        ra, rb = a.run(1)[0], b.run(1)[0]
        assert ra.attempts == rb.attempts == 1
        assert np.array_equal(a.vx, b.vx) and np.array_equal(a.vy, b.vy) and np.array_equal(a.vz, b.vz)
        assert (ra.collisions, ra.R0, ra.n_th, ra.m_state_after) == (rb.collisions, rb.R0, rb.n_th, rb.m_state_after)


@pytest.mark.parametrize("alpha,eps", [(0.0, 0.05), (1.0, 0.3)])
def test_no_discarded_work(orc, alpha, eps):
    vx, vy, vz = W.bkw(6000, 0.6, seed=4)
    kw = dict(eps=eps, dt=0.05, alpha=alpha, m_init=2, m_cap=16, **FORCE)
    plain = orc.Instance(vx, vy, vz, trunc=orc.ADAPTIVE, **kw)
    reuse = orc.Instance(vx, vy, vz, trunc=orc.ADAPTIVE_REUSE, **kw)
    rp, rr = plain.run(1)[0], reuse.run(1)[0]
    assert rp.attempts == rr.attempts == 4  # depths 2, 4, 8, 16
    assert rr.work_collisions == rr.collisions
    assert rp.work_collisions > rp.collisions
    assert rr.work_collisions < rp.work_collisions
    assert rr.m_used == rp.m_used == 16 and rr.N0 == rp.N0


@pytest.mark.parametrize("x,m", [(1.204, 8), (0.693, 4)])
def test_stress_decay_of_the_final_depth(orc, x, m):
    n, reps = 20000, 24
    tau = _tau(x)
    num = den = 0.0
    for r in range(reps):
        vx, vy, vz = W.bkw(n, 0.6, seed=10, stream=r)
        vx = vx * 1.3  # anisotropic: P_xx != T
        inst = orc.Instance(vx, vy, vz, eps=1.0, dt=x, trunc=orc.ADAPTIVE_REUSE, m_init=2, m_cap=m, uid=r,
                            **FORCE)
        a = inst.moments()[0]
        inst.run(1)
        assert inst.last[0].attempts == int(math.log2(m))  # 2 -> ... -> m
        b = inst.moments()[0]
        num += b[5] - b[4]
        den += a[5] - a[4]
    assert num / den == pytest.approx(r2(tau, m), abs=0.02)
    assert num / den - r2(tau, m // 2) > 0.02  # not the law of a shallower depth


def test_fourth_moment_decay_of_the_final_depth(orc):
    x, m, n, reps = 1.204, 8, 20000, 24
    tau = _tau(x)
    num = den = 0.0
    for r in range(reps):
        vx, vy, vz = W.bkw(n, 0.6, seed=11, stream=r)
        inst = orc.Instance(vx, vy, vz, eps=1.0, dt=x, trunc=orc.ADAPTIVE_REUSE, m_init=2, m_cap=m, uid=r,
                            **FORCE)
        a = inst.moments()[0]
        inst.run(1)
        b = inst.moments()[0]
        num += b[8] - 15 * b[4] ** 2
        den += a[8] - 15 * a[4] ** 2
    assert num / den == pytest.approx(r4(tau, m), abs=0.03)


@pytest.mark.parametrize("alpha,eps", [(0.0, 0.05), (1.0, 0.3), (1.0, 0.05)])
def test_conservation(orc, alpha, eps):
    vx, vy, vz = W.bimaxwellian(4000, seed=6)
    inst = orc.Instance(vx, vy, vz, eps=eps, alpha=alpha, trunc=orc.ADAPTIVE_REUSE, m_init=2, m_cap=64)
    s = float(np.abs(inst.vx).sum() + np.abs(inst.vy).sum() + np.abs(inst.vz).sum())
    p0 = np.array([inst.vx.sum(), inst.vy.sum(), inst.vz.sum()])
    e0 = float((inst.vx**2 + inst.vy**2 + inst.vz**2).sum())
    redo = 0
    for _ in range(5):
        redo += inst.run(1)[0].attempts > 1
    p1 = np.array([inst.vx.sum(), inst.vy.sum(), inst.vz.sum()])
    e1 = float((inst.vx**2 + inst.vy**2 + inst.vz**2).sum())
    assert redo > 0  # some step really extended a rejected attempt
    assert np.abs(p1 - p0).max() <= 1e-12 * s
    assert abs(e1 - e0) <= 1e-12 * e0


def test_rejects_unknown_truncation_and_tree_shape_with_reuse(orc):
    vx, vy, vz = W.bimaxwellian(100, seed=1)
    with pytest.raises(RuntimeError):
        orc.Instance(vx, vy, vz, trunc=4).run(1)
    with pytest.raises(RuntimeError):
        orc.Instance(vx, vy, vz, trunc=orc.ADAPTIVE_REUSE, wb=orc.WB_MIN, wb_mmax=3).run(1)
