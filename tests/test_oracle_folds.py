"""The fold rule of the tree schedule (reading R6): while the trees ask for more
leaves than the cell holds, the deepest level is folded into the remainder and
the trees are rebuilt.  The leaves needed, R0(m), do not decrease with the depth
m of the trees (same split sizes below m, same keyed sub-level choices), so the
depth that the downward scan stops at is also the largest m with R0(m) <= n,
which a bisection finds in a logarithmic number of rebuilds.

The lemma is checked here by brute force with an integer tree pass written
from the level-order rule alone (requests counted per level, collisions
ceil(R_l/2) + ceil(max(0, N_l - R_l mod 2)/2), sub-level choices from Philox
TREE draws), and its consequence against the oracle's own scan.
"""
import numpy as np
import pytest

TAG_TREE = 3


class Choices:
    """Sub-level choice j of collision c of level l: one Philox block per four
    collisions, j = floor(w * l / 2^32)."""

    def __init__(self, orc, seed, uid, cell, step):
        self.orc, self.key, self.cell, self.step = orc, (seed, uid), cell, step
        self.cache = {}

    def __call__(self, l, c):
        k = (l, c >> 2)
        if k not in self.cache:
            self.cache[k] = self.orc.philox([c >> 2, (TAG_TREE << 24) | l, self.cell, self.step], self.key)
        return (int(self.cache[k][c & 3]) * l) >> 32


def leaves_needed(N, me, choose):
    """R0 of trees of depth me over split sizes N[1..me] (no folding)."""
    R = [0] * (me + 2)
    for l in range(me, 0, -1):
        odd = R[l] & 1
        Nl = int(N[l])
        own = (Nl - odd + 1) // 2 if Nl > odd else 0
        for c in range((R[l] + 1) // 2 + own):
            j = choose(l, c)
            R[j] += 1
            R[l - 1 - j] += 1
    return R[0]


CASES = [(n, q, s) for n in (17, 60, 150) for q in (0.02, 0.08, 0.3) for s in range(4)]


@pytest.mark.parametrize("n,q,s", CASES)
def test_leaves_needed_grow_with_depth(orc, n, q, s):
    seed, uid, cell, step, m_cap = 3, 40 + s, 0, s, 2048
    N, me = orc.split(seed, uid, cell, step, n, q, m_cap)
    choose = Choices(orc, seed, uid, cell, step)
    R0 = [leaves_needed(N, m, choose) for m in range(me + 1)]
    assert all(a <= b for a, b in zip(R0, R0[1:])), R0
    # the downward scan of the fold rule and the largest depth that fits agree
    scan = me
    while R0[scan] > n:
        scan -= 1
    fits = max(m for m in range(me + 1) if R0[m] <= n)
    assert scan == fits
    t = orc.tree(seed, uid, cell, step, n, q, m_cap)
    assert t["me"] == scan and t["R0"] == R0[scan]


def test_folding_happens_in_these_cases(orc):
    """The cases above include deep splits whose trees need folding."""
    folded = 0
    for n, q, s in CASES:
        N, me = orc.split(3, 40 + s, 0, s, n, q, 2048)
        t = orc.tree(3, 40 + s, 0, s, n, q, 2048)
        folded += t["me"] < me
    assert folded >= 10
