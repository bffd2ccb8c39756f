"""The VHS majorant raised level by level (Remark 4.1, reading R18) in the oracle.

The step's bound sigma(2 dv) holds for every pair of pre-step velocities, but
collisions move velocities away from the mean (by up to a factor sqrt(2) per
collision), so pairs of deeper levels can exceed it; the fixed bound counts
them as violations and accepts them with probability 1.  With the bound of
level l taken from the largest distance to the mean among the velocities that
level l can draw from (the pre-step ones and the outputs of levels below l),
|v_a - v_b| <= |v_a - mean| + |v_b - mean| <= 2 dv_l for every pair, so no
violation can occur.  Pins:

  * no violations, in cases where the fixed bound has many;
  * Maxwell molecules (no bound used) and depth 1 (only the step's bound):
    identical to the fixed bound, bitwise;
  * the recorded bound is at least the step's bound on the 20-bit grid;
  * exact conservation.
"""
import numpy as np
import pytest

import workloads as W


def run(orc, v, majorant, eps, alpha=1.0, trunc=None, m=24, uid=0, steps=1, n=None):
    vx, vy, vz = v
    n = len(vx)
    inst = orc.Instance(vx, vy, vz, eps=eps, dt=0.05, alpha=alpha, trunc=orc.FIXED if trunc is None else trunc,
                        m_init=m, m_cap=64, uid=uid, weight=1.0 / n, majorant=majorant)
    inst.run(steps)
    return inst


@pytest.mark.parametrize("eps", [0.02, 0.05, 0.1])
def test_level_majorant_has_no_violations(orc, eps):
    """Velocities on a sphere around the mean: outputs of collisions reach up to
    sqrt(2) dv from the mean, and pairs of them exceed the step's bound."""
    fixed_viol = 0
    for s in range(6):
        v = W.shell(2000, seed=31, stream=s)
        a = run(orc, v, orc.MAJ_STEP, eps, uid=s)
        b = run(orc, v, orc.MAJ_LEVEL, eps, uid=s)
        fixed_viol += int(a.last[0].violations)
        assert int(b.last[0].violations) == 0
        assert b.last[0].collisions == a.last[0].collisions  # same schedule (same split and trees)
        assert b.last[0].g >= a.last[0].g
    assert fixed_viol > 20  # the fixed bound is exceeded in these cases


def test_level_majorant_equals_fixed_for_maxwell_molecules(orc):
    v = W.bkw(3000, 0.6, seed=32)
    a = run(orc, v, orc.MAJ_STEP, 0.01, alpha=0.0, steps=3)
    b = run(orc, v, orc.MAJ_LEVEL, 0.01, alpha=0.0, steps=3)
    for k in ("vx", "vy", "vz"):
        assert np.array_equal(getattr(a, k), getattr(b, k))


def test_level_majorant_equals_fixed_at_depth_one(orc):
    v = W.bimaxwellian(3000, seed=33)
    a = run(orc, v, orc.MAJ_STEP, 0.02, m=1, steps=3)
    b = run(orc, v, orc.MAJ_LEVEL, 0.02, m=1, steps=3)
    for k in ("vx", "vy", "vz"):
        assert np.array_equal(getattr(a, k), getattr(b, k))


def test_recorded_bound_is_at_least_the_steps(orc):
    v = W.shell(5000, seed=34)
    vx, vy, vz = v
    d = np.stack(v, 1) - np.stack(v, 1).mean(0)
    g0 = orc.grid_up(2.0 * np.sqrt((d * d).sum(1).max()))
    b = run(orc, v, orc.MAJ_LEVEL, 0.05, uid=4)
    assert b.last[0].g > g0  # raised: outputs went beyond the pre-step dv
    a = run(orc, v, orc.MAJ_STEP, 0.05, uid=4)
    assert a.last[0].g == g0


@pytest.mark.parametrize("trunc", ["fixed", "adaptive", "natural"])
def test_level_majorant_conserves(orc, trunc):
    tr = {"fixed": orc.FIXED, "adaptive": orc.ADAPTIVE, "natural": orc.NATURAL}[trunc]
    v = W.shell(3000, seed=35)
    inst = orc.Instance(*v, eps=0.05, dt=0.05, alpha=1.0, trunc=tr, m_init=4, m_cap=64, weight=1.0 / 3000,
                        majorant=orc.MAJ_LEVEL)
    for _ in range(4):
        p0 = np.array([inst.vx.sum(), inst.vy.sum(), inst.vz.sum()])
        e0 = (inst.vx ** 2 + inst.vy ** 2 + inst.vz ** 2).sum()
        inst.run(1)
        p1 = np.array([inst.vx.sum(), inst.vy.sum(), inst.vz.sum()])
        e1 = (inst.vx ** 2 + inst.vy ** 2 + inst.vz ** 2).sum()
        assert np.abs(p1 - p0).max() <= 1e-13 * np.abs(np.stack([inst.vx, inst.vy, inst.vz])).sum()
        assert abs(e1 - e0) <= 1e-13 * e0
        assert int(inst.last[0].violations) == 0


def test_level_majorant_rejected_with_reuse_or_tree_shape(orc):
    v = W.bimaxwellian(500, seed=36)
    for kw in (dict(trunc=orc.ADAPTIVE_REUSE), dict(trunc=orc.FIXED, wb=orc.WB_MIN, wb_mmax=2)):
        inst = orc.Instance(*v, eps=0.05, dt=0.05, alpha=1.0, m_init=2, m_cap=64, weight=1.0 / 500,
                            majorant=orc.MAJ_LEVEL, **kw)
        with pytest.raises(RuntimeError):
            inst.run(1)
