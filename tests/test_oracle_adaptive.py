"""Pins of the oracle's adaptive depth (Sec. 4.3): the indicator E1 and the
halve / keep / recompute rule, against what the mathematics fixes.

E1 = |S^{n+1,m} - S^n| / |S^n| with S = P_xx per unit mass and the thermalized
part entering through its expected value (energy of the removed set over 3 plus
the shift of its mean).  Pins:

  * eps -> 0 (every particle thermalized): S^{n+1,m} is the temperature T of
    the cell exactly, so E1 = |T - S^n| / S^n;
  * eps -> infinity (nothing collides): E1 = 0;
  * Maxwell molecules, ensemble mean: the Wild sum truncated at depth m relaxes
    the traceless stress by r2(tau, m) = (1 - tau) sum_{k<=m} C(2k,k) 4^-k tau^k
    in expectation (the thermalized part has no traceless stress), so
    E[E1] = (1 - r2(tau, m)) (S^n - T) / S^n at the accepted depth, when the
    anisotropy is large against the sampling noise;
  * the decision: E1 below delta1 halves the next depth (floor, at least 1);
    between delta1 and delta2 keeps it; above delta2 recomputes at twice the
    depth until m_cap, or stops when the split left no remainder.
"""
import math

import numpy as np
import pytest
from scipy import special

import workloads as W


def r2(tau, m):
    """Decay of the traceless stress per step for Maxwell molecules (the generating
    function (1-tau)^(-1/2) of the Wild sum, truncated after tau^m)."""
    return (1 - tau) * sum(math.exp(special.gammaln(k + 0.5) - special.gammaln(0.5) - special.gammaln(k + 1))
                           * tau**k for k in range(m + 1))


def drifting_bimaxwellian(n, seed, stream, drift=0.7):
    """Bi-Maxwellian along x (P_xx = 2, T = 4/3 per unit mass) moving with +drift
    along x: a mean that the indicator must subtract."""
    vx, vy, vz = W.bimaxwellian(n, seed=seed, stream=stream)
    return vx + drift, vy, vz


def cell_S_T(vx, vy, vz):
    """S = P_xx per unit mass and T of the data (plain numpy, FP64)."""
    ux, uy, uz = vx.mean(), vy.mean(), vz.mean()
    S = float(((vx - ux) ** 2).mean())
    T = float((((vx - ux) ** 2) + ((vy - uy) ** 2) + ((vz - uz) ** 2)).mean() / 3.0)
    return S, T


def test_indicator_all_thermalized_is_temperature_gap(orc):
    """eps -> 0: q = 0, every particle goes to the Maxwellian, the expected
    stress after the step is T, so E1 = |T - S| / S exactly (up to rounding)."""
    for stream, drift in ((0, 0.0), (1, 0.7), (2, -2.5)):
        vx, vy, vz = drifting_bimaxwellian(3000, seed=21, stream=stream, drift=drift)
        S, T = cell_S_T(vx, vy, vz)
        inst = orc.Instance(vx, vy, vz, eps=1e-7, dt=0.05, trunc=orc.ADAPTIVE, m_init=2, m_cap=64,
                            delta1=10.0, delta2=20.0, weight=1.0 / 3000)
        rec = inst.run(1)[0]
        assert rec.n_th == 3000 and rec.R0 == 0 and rec.N0 == 0
        assert rec.E1 == pytest.approx(abs(T - S) / S, rel=1e-12, abs=1e-14)


def test_indicator_collisionless_is_zero(orc):
    vx, vy, vz = drifting_bimaxwellian(2000, seed=22, stream=0)
    inst = orc.Instance(vx, vy, vz, eps=1e12, dt=0.05, trunc=orc.ADAPTIVE, m_init=2, m_cap=64,
                        weight=1.0 / 2000)
    rec = inst.run(1)[0]
    assert rec.N0 == 2000 and rec.E1 <= 1e-13 and rec.attempts == 1  # zero up to the sums' rounding
    assert rec.m_state_after == 1  # E1 < delta1: the depth halves (floor, at least 1)


@pytest.mark.parametrize("x,m_init,m_cap", [(0.693, 2, 4), (1.204, 1, 2), (2.303, 4, 8), (0.357, 1, 1)])
def test_indicator_mean_follows_stress_decay(orc, x, m_init, m_cap):
    """Maxwell molecules on drifting bi-Maxwellian data: the indicator's ensemble
    mean equals (1 - r2(tau, m)) (S - T) / S at the accepted depth.  The data are
    far enough from equilibrium that E1 > delta2 at every depth below m_cap, so
    the accepted depth is m_cap whatever the noise (no selection by E1)."""
    n, reps = 20000, 32
    tau = 1.0 - math.exp(-x)
    d = []
    for r in range(reps):
        vx, vy, vz = drifting_bimaxwellian(n, seed=23, stream=r)
        S, T = cell_S_T(vx, vy, vz)
        inst = orc.Instance(vx, vy, vz, eps=1.0, dt=x, trunc=orc.ADAPTIVE, m_init=m_init, m_cap=m_cap,
                            uid=r, weight=1.0 / n)
        rec = inst.run(1)[0]
        assert rec.m_used == m_cap
        assert rec.q == pytest.approx(1.0 - tau, rel=1e-12)
        d.append(rec.E1 - (1.0 - r2(tau, m_cap)) * (S - T) / S)
    d = np.array(d)
    expect = (1.0 - r2(tau, m_cap)) * (2.0 - 4.0 / 3.0) / 2.0
    assert expect > 0.05  # the signal is far above delta2 and above the noise
    assert abs(d.mean()) <= 3.0 * d.std(ddof=1) / math.sqrt(reps) + 1e-4 * expect, (d.mean(), d.std())


def test_decision_rule_branches(orc):
    """The three branches of Sec. 4.3 with thresholds placed around an indicator
    of about 0.1 (tau = 0.5 at depth 4 on bi-Maxwellian data, n = 20000: its
    noise is about 0.003): below delta1 the next depth halves, between the
    thresholds it stays, above delta2 the step is recomputed at twice the depth
    up to m_cap, and the accepted result equals a run at that fixed depth."""
    n = 20000
    vx, vy, vz = drifting_bimaxwellian(n, seed=24, stream=0)
    common = dict(eps=1.0, dt=0.693, weight=1.0 / n, m_cap=16)
    # E1 < delta1: accept, next depth floor(m / 2)
    for m_init, after in ((4, 2), (3, 1), (1, 1)):
        inst = orc.Instance(vx, vy, vz, trunc=orc.ADAPTIVE, m_init=m_init, delta1=0.5, delta2=0.9, **common)
        rec = inst.run(1)[0]
        assert (rec.attempts, rec.m_used, rec.m_state_after) == (1, m_init, after)
        assert 0.02 < rec.E1 < 0.5
    # delta1 <= E1 <= delta2: accept, keep the depth
    inst = orc.Instance(vx, vy, vz, trunc=orc.ADAPTIVE, m_init=4, delta1=0.01, delta2=0.9, **common)
    rec = inst.run(1)[0]
    assert (rec.attempts, rec.m_used, rec.m_state_after) == (1, 4, 4)
    # E1 > delta2: recompute at 2m until m_cap (4 -> 8 -> 16), keep m_cap
    inst = orc.Instance(vx, vy, vz, trunc=orc.ADAPTIVE, m_init=4, delta1=0.001, delta2=0.002, **common)
    rec = inst.run(1)[0]
    assert (rec.attempts, rec.m_used, rec.m_state_after) == (3, 16, 16)
    fixed = orc.Instance(vx, vy, vz, trunc=orc.FIXED, m_init=16, **common)
    fixed.run(1)
    assert np.array_equal(inst.vx, fixed.vx) and np.array_equal(inst.vy, fixed.vy)
    # a depth that is not a power of two of m_init: 3 -> 6 -> 12 -> 16 (capped)
    inst = orc.Instance(vx, vy, vz, trunc=orc.ADAPTIVE, m_init=3, delta1=0.001, delta2=0.002, **common)
    rec = inst.run(1)[0]
    assert (rec.attempts, rec.m_used, rec.m_state_after) == (4, 16, 16)


def test_decision_stops_when_split_has_no_remainder(orc):
    """A split that used up every particle before depth m has nothing to gain from
    a deeper attempt: the step is accepted even with E1 above delta2."""
    n = 400
    seen = 0
    for s in range(40):
        vx, vy, vz = drifting_bimaxwellian(n, seed=25, stream=s)
        # tau about 0.1: the split runs dry after a few levels
        inst = orc.Instance(vx, vy, vz, eps=1.0, dt=0.105, trunc=orc.ADAPTIVE, m_init=8, m_cap=64,
                            delta1=1e-12, delta2=2e-12, uid=s, weight=1.0 / n)
        rec = inst.run(1)[0]
        if rec.m_eff < 8:  # the split stopped with no remainder
            seen += 1
            assert rec.attempts == 1 and rec.m_state_after == 8 and rec.n_th == 0
        else:
            assert rec.attempts > 1 or rec.E1 <= 2e-12
    assert seen >= 5


def test_decision_zero_stress_accepts(orc):
    """S^n = 0 (every particle with the same x-velocity): nothing to measure the
    change against; the step is accepted at its depth."""
    n = 500
    g = np.random.default_rng(3)
    vx = np.full(n, 0.25)
    vy, vz = g.standard_normal(n), g.standard_normal(n)
    inst = orc.Instance(vx, vy, vz, eps=0.5, dt=0.05, trunc=orc.ADAPTIVE, m_init=4, m_cap=64,
                        delta1=1e-9, delta2=2e-9, weight=1.0 / n)
    rec = inst.run(1)[0]
    assert rec.attempts == 1 and rec.m_state_after == 4


def test_no_recompute_when_deeper_levels_stay_empty(orc):
    """A recompute at a greater depth cannot change the step when the split,
    continued from the remainder, puts no particle in any level up to m_cap:
    the deeper trees are those of depth m.  Then the step is accepted at once
    and keeps its depth, with the velocities a run at m_cap would give."""
    n = 2000
    vx, vy, vz = drifting_bimaxwellian(n, seed=26, stream=0)
    # eps -> 0: q = 0, every level empty, everything thermalized; E1 = |T - S|/S > delta2
    for m_init in (1, 2, 5):
        inst = orc.Instance(vx, vy, vz, eps=1e-7, dt=0.05, trunc=orc.ADAPTIVE, m_init=m_init, m_cap=64,
                            weight=1.0 / n)
        rec = inst.run(1)[0]
        assert rec.E1 > 0.1 and (rec.attempts, rec.m_used, rec.m_state_after) == (1, m_init, m_init)
        deep = orc.Instance(vx, vy, vz, eps=1e-7, dt=0.05, trunc=orc.FIXED, m_init=64, m_cap=64, weight=1.0 / n)
        deep.run(1)
        assert np.array_equal(inst.vx, deep.vx) and np.array_equal(inst.vz, deep.vz)


def test_recompute_only_when_a_deeper_level_fills(orc):
    """Small q rem: whether the step is recomputed depends on the keyed draws of
    the deeper levels alone.  Either it is accepted at once and equals the run
    at m_cap bitwise (the deeper levels stayed empty), or it is recomputed."""
    n = 3000
    seen = {True: 0, False: 0}
    for s in range(30):
        vx, vy, vz = drifting_bimaxwellian(n, seed=27, stream=s)
        # tau close to 1 with depth 4 of 8: a remainder of about q^... particles
        kw = dict(eps=1.0, dt=9.0, alpha=0.0, uid=s, weight=1.0 / n, m_cap=8)
        a = orc.Instance(vx, vy, vz, trunc=orc.ADAPTIVE, m_init=4, delta1=1e-12, delta2=2e-12, **kw)
        rec = a.run(1)[0]
        if rec.attempts == 1:
            assert rec.m_state_after == 4
            b = orc.Instance(vx, vy, vz, trunc=orc.FIXED, m_init=8, **kw)
            b.run(1)
            assert np.array_equal(a.vx, b.vx) and np.array_equal(a.vy, b.vy)
        seen[rec.attempts == 1] += 1
    assert seen[True] >= 3 and seen[False] >= 3
