"""Pins of the oracle's tree-shape truncation (TRMC-WB, Sec. 4.4).

* The length rule against Table 1: of the 429 shapes of a 7-collision tree the
  balanced one is the only one of lengths (3, 3) under definitions def:2 and
  def:3, and a shape of lengths (2, 43/16) exists; definition def:1 gives 7.
* The level-order lengths of every final against the explicit per-sample tree
  of Alg. 4.5 (the preorder list of sub-level choices), evaluated in exact
  rational arithmetic.
* Invariants of the step: m_max at or above the depth changes nothing; the
  thermalized finals are those longer than m_max; momentum and energy are kept.
"""
from fractions import Fraction
from functools import lru_cache

import numpy as np
import pytest

import workloads as W


# ----------------------------------------------------------------------------
# Table 1: lengths of 7-collision trees
# ----------------------------------------------------------------------------
@lru_cache(None)
def _shapes(k):
    """Every tree of k collisions: a leaf for k = 0, else (left, right) with
    sizes j and k - 1 - j (Alg. 4.5: j uniform in 0..k-1, h = k - 1 - j)."""
    if k == 0:
        return (None,)
    return tuple((a, b) for j in range(k) for a in _shapes(j) for b in _shapes(k - 1 - j))


def _length(t, kind, orc):
    if t is None:
        return 0.0
    return orc.wb_len(_length(t[0], kind, orc), _length(t[1], kind, orc), kind)


def _size(t):
    return 0 if t is None else 1 + _size(t[0]) + _size(t[1])


def test_table1_tree_lengths(orc):
    shapes = _shapes(7)
    assert len(shapes) == 429  # Catalan number C_7
    lens = [(_length(t, orc.WB_MIN, orc), _length(t, orc.WB_MEAN, orc)) for t in shapes]
    # def:1, the size of the tree, is 7 for both trees of Table 1
    assert all(_size(t) == 7 for t in shapes)
    # left tree of Table 1: 3 under def:2 and def:3, and only the balanced tree has it
    balanced = (((None, None), (None, None)), ((None, None), (None, None)))
    assert _length(balanced, orc.WB_MIN, orc) == 3.0 and _length(balanced, orc.WB_MEAN, orc) == 3.0
    assert [i for i, lv in enumerate(lens) if lv == (3.0, 3.0)] == [shapes.index(balanced)]
    # right tree of Table 1: 2 under def:2 and 43/16 under def:3
    assert (2.0, 43 / 16) in lens
    # def:2 never exceeds def:3, which never exceeds def:1
    assert all(a <= b <= 7 for a, b in lens)


# ----------------------------------------------------------------------------
# Level-order lengths against the explicit trees of Alg. 4.5
# ----------------------------------------------------------------------------
def _path(t, level, out, path):
    """Preorder list of Alg. 4.5 for output `out` of level `level`: k, then for
    k > 0 the sub-level choices j, h followed by the two subtrees."""
    path.append(level)
    if level == 0:
        return
    c = out // 2
    cid = int(t["first"][level]) + c
    j = int(t["j"][cid])
    h = level - 1 - j
    path.append(j)
    path.append(h)
    _path(t, j, int(t["rA"][cid]), path)
    _path(t, h, int(t["rB"][cid]), path)


def _eval_path(path, pos, kind):
    """Length of the tree whose preorder list starts at pos (exact rationals)."""
    k = path[pos]
    if k == 0:
        return Fraction(0), pos + 1, 0
    j, h = path[pos + 1], path[pos + 2]
    a, p, sa = _eval_path(path, pos + 3, kind)
    b, p, sb = _eval_path(path, p, kind)
    size = 1 + sa + sb
    assert sa == j and sb == h  # a sample of f_k is made by exactly k collisions
    L = 1 + (min(a, b) if kind == 1 else (a + b) / 2)
    return L, p, size


@pytest.mark.parametrize("n,q,m", [(3000, 0.05, 64), (20000, 0.1, 12), (800, 0.01, 40)])
@pytest.mark.parametrize("kind", [1, 2])
def test_final_lengths_match_explicit_trees(orc, n, q, m, kind):
    t = orc.tree(7, 3, 1, 2, n, q, m, kind)
    finals = []
    for lv in range(1, t["me"] + 1):
        for o in range(int(t["R"][lv]), 2 * int(t["C"][lv])):
            finals.append((lv, o))
    assert len(finals) == t["R0"] == len(t["finlen"])
    assert t["me"] >= 8  # deep enough for lengths to differ from the level
    for (lv, o), got in zip(finals, t["finlen"]):
        path = []
        _path(t, lv, o, path)
        L, end, size = _eval_path(path, 0, kind)
        assert end == len(path) and size == lv
        if kind == 1:
            assert got == float(L)
        else:
            assert abs(got - float(L)) <= 1e-12 * float(L)
        for mmax in range(1, 10):
            if abs(float(L) - mmax) > 1e-9:
                assert (got > mmax) == (L > mmax)


# ----------------------------------------------------------------------------
# The step with tree-shape truncation
# ----------------------------------------------------------------------------
def _inst(orc, n, wb, mmax, m=16, alpha=0.0, eps=0.05, seed=4, uid=9):
    vx, vy, vz = W.bimaxwellian(n, seed=seed, stream=1)
    return orc.Instance(vx, vy, vz, seed=seed, uid=uid, eps=eps, alpha=alpha, trunc=orc.FIXED, m_init=m,
                        m_cap=64, wb=wb, wb_mmax=mmax)


@pytest.mark.parametrize("wb", [1, 2])
def test_mmax_at_depth_changes_nothing(orc, wb):
    """Lengths never exceed the level (def:2 <= def:3 <= def:1), so m_max >= m
    leaves the step identical to the plain one."""
    a = _inst(orc, 4000, orc.WB_OFF, 5)
    b = _inst(orc, 4000, wb, 16)
    ra, rb = a.run(3), b.run(3)
    assert np.array_equal(a.vx, b.vx) and np.array_equal(a.vy, b.vy) and np.array_equal(a.vz, b.vz)
    assert rb[0].wb_th == 0 and ra[0].n_th == rb[0].n_th and ra[0].collisions == rb[0].collisions


@pytest.mark.parametrize("wb,mmax,alpha,eps", [(1, 2, 0.0, 0.02), (2, 2, 1.0, 0.2), (2, 3, 1.0, 0.1), (1, 2, 1.0, 0.1)])
def test_thermalized_finals_are_the_long_trees(orc, wb, mmax, alpha, eps):
    # hard spheres: mu = rho (2 dv) is about ten times Maxwell's, so a larger eps
    # gives trees of similar depth
    plain = _inst(orc, 6000, orc.WB_OFF, mmax, alpha=alpha, eps=eps)
    inst = _inst(orc, 6000, wb, mmax, alpha=alpha, eps=eps)
    rp, rec = plain.run(1)[0], inst.run(1)[0]
    t = orc.tree(inst.seed, inst.uid, 0, 0, 6000, rec.q, 16, wb)
    expect = int(np.sum(t["finlen"] > mmax))
    assert expect > 0
    assert rec.wb_th == expect
    assert rec.n_th == rp.n_th + expect
    assert rec.collisions == rp.collisions and rec.R0 == rp.R0 and rec.N0 == rp.N0
    # unchanged and tree-final slots agree with the plain step; the thermalized
    # ones (a larger set, so a different rescale) all differ
    same = (plain.vx == inst.vx) & (plain.vy == inst.vy) & (plain.vz == inst.vz)
    assert int((~same).sum()) == rec.n_th


@pytest.mark.parametrize("wb", [1, 2])
def test_step_conserves_momentum_and_energy(orc, wb):
    inst = _inst(orc, 5000, wb, 2, alpha=1.0, eps=0.2)
    p0 = np.array([inst.vx.sum(), inst.vy.sum(), inst.vz.sum()])
    e0 = float((inst.vx**2 + inst.vy**2 + inst.vz**2).sum())
    s = float(np.abs(inst.vx).sum() + np.abs(inst.vy).sum() + np.abs(inst.vz).sum())
    th = 0
    for _ in range(4):
        th += inst.run(1)[0].wb_th
    p1 = np.array([inst.vx.sum(), inst.vy.sum(), inst.vz.sum()])
    e1 = float((inst.vx**2 + inst.vy**2 + inst.vz**2).sum())
    assert th > 0
    assert np.abs(p1 - p0).max() <= 1e-12 * s
    assert abs(e1 - e0) <= 1e-12 * e0


def test_rejects_adaptive_and_zero_mmax(orc):
    vx, vy, vz = W.bimaxwellian(100, seed=1, stream=1)
    bad = orc.Instance(vx, vy, vz, trunc=orc.ADAPTIVE, wb=orc.WB_MIN, wb_mmax=5)
    with pytest.raises(RuntimeError):
        bad.run(1)
    bad = orc.Instance(vx, vy, vz, trunc=orc.FIXED, wb=orc.WB_MEAN, wb_mmax=0)
    with pytest.raises(RuntimeError):
        bad.run(1)
