"""Depth-first TRMC-R sampler in the order of Alg. 4.3 (test infrastructure only).

This is a second, independent rendering of the recursive collision step used
only as a statistical twin of the level-order oracle: it follows the paper's
depth-first order (levels m..1, recursive sampling of lower densities on demand,
one stored twin per level reused by the next request), with its own random
numbers from numpy.  Counts and moments of the two must agree in law, not
realization by realization.

Pool exhaustion, which the paper does not discuss, is handled as in the oracle:
leaves first come from the particles not kept unchanged, then from the kept
block; the depth is lowered by one while even that is not enough.
"""
from __future__ import annotations

import math
import sys

import numpy as np


def _iround(y: float, u: float) -> int:
    f = math.floor(y)
    return int(f) + (1 if u < y - f else 0)


def _collide(a, b, g, alpha, gen):
    q = a - b
    qn = math.sqrt(float(q @ q))
    if alpha != 0.0:
        s = qn ** alpha
        if not (gen.random() * g < s):
            return a.copy(), b.copy(), False
    ct = 2.0 * gen.random() - 1.0
    st = math.sqrt(max(0.0, 1.0 - ct * ct))
    phi = 2.0 * math.pi * gen.random()
    sig = np.array([math.cos(phi) * st, math.sin(phi) * st, ct])
    c = 0.5 * (a + b)
    return c + 0.5 * qn * sig, c - 0.5 * qn * sig, True


def step(v: np.ndarray, q: float, m: int, gen: np.random.Generator, alpha: float = 0.0, g: float = 1.0):
    """One collision step of one cell, depth-first.  Returns (new v, collisions, thermalized)."""
    n = len(v)
    if n < 2:
        return v.copy(), 0, 0
    sys.setrecursionlimit(max(10000, 4 * m + 100))
    # Alg. 4.2
    N = [0] * (m + 2)
    N[0] = _iround(q * n, gen.random())
    rem = n - N[0]
    k = 0
    while rem > 0 and k < m:
        k += 1
        N[k] = _iround(q * rem, gen.random())
        rem -= N[k]
    me = k
    N[me + 1] = rem
    order = gen.permutation(n)
    while True:
        Nrem = list(N)
        stored = [[] for _ in range(me + 2)]
        leaves_used = []
        finals = {l: [] for l in range(1, me + 1)}
        ncoll = [0]
        pool = list(order[N[0]:]) + list(order[:N[0]][::-1])
        ok = [True]

        def leaf():
            if len(leaves_used) >= n:
                ok[0] = False
                return np.zeros(3)
            s = pool[len(leaves_used)]
            leaves_used.append(s)
            return v[s].copy()

        def get(kk):
            if kk == 0:
                return leaf()
            if stored[kk]:
                Nrem[kk] += 1
                return stored[kk].pop()
            a, b = pair(kk)
            stored[kk].append(b)
            Nrem[kk] -= 1
            return a

        def pair(l):
            kk = int(gen.integers(0, l))
            x = get(kk)
            y = get(l - 1 - kk)
            ncoll[0] += 1
            a, b, _ = _collide(x, y, g, alpha, gen)
            return a, b

        for l in range(me, 0, -1):
            while Nrem[l] > 0:
                a, b = pair(l)
                finals[l] += [a, b]
                Nrem[l] -= 2
            finals[l] += stored[l]
            stored[l] = []
        if ok[0]:
            break
        N[me] += N[me + 1]
        me -= 1
    out = v.copy()
    fin = [f for l in range(1, me + 1) for f in finals[l]]
    assert len(fin) == len(leaves_used)
    for s, f in zip(leaves_used, fin):
        out[s] = f
    P = n - N[0]
    th = [s for s in pool[len(leaves_used):P]] if len(leaves_used) < P else []
    if len(th) >= 2:
        old = v[th]
        ur = old.mean(axis=0)
        E = float(((old - ur) ** 2).sum())
        z = gen.standard_normal((len(th), 3))
        zc = z - z.mean(axis=0)
        out[th] = ur + math.sqrt(E / float((zc ** 2).sum())) * zc
    return out, ncoll[0], len(th)
