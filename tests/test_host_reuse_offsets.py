"""Host model of the index arithmetic of the whole-cell step with the adaptive
depth that keeps rejected attempts (Sec. 4.3).

The kernel's per-cell scratch and LDS offsets are restated here from its own
layout rules (collision capacity 4n + 256, level outputs 2 per collision, finals
and leaves by rank in arrays of n records, level arrays of m_cap + 2 entries, the
draw-offset array after the level arrays of the workgroup's groups) and checked
against the integer outline of every attempt that the oracle makes on the
benchmark's reuse workload: leaf and final ranks of kept attempts against n,
level outputs against their capacity, tree indices against the collision
capacity, draw offsets against 32 bits, and every LDS offset against the
dynamic LDS the runtime allocates, for workgroups of 256 and 512 threads with
groups of 64 and of the whole workgroup.
"""
import numpy as np
import pytest

import oracle as orc
import workloads as W


def coll_cap(n):
    return 4 * n + 256


def scratch_bytes(n, sz):
    """Bytes the runtime reserves for a cell of n particles (element size sz)."""
    bpp = (56 + 40 * sz + 15) // 16 * 16
    cpc = ((256 * (12 + 8 * sz) + 195 + 255) // 256) * 256
    return bpp * n + cpc


def scratch_used(n, sz):
    """Bytes the kernel's layout of one cell spans: role, fwd (u32), leaf and fin
    (4-component records), j / rA / rB (u32 per collision), outputs (2 records
    per collision)."""
    a16 = lambda b: (b + 15) // 16 * 16
    cap = coll_cap(n)
    return a16(4 * n) * 2 + 2 * 4 * sz * n + 3 * a16(4 * cap) + 2 * cap * 4 * sz


def lds_check(nt, g, m_cap):
    """Dynamic LDS of a reuse launch against the largest offset a group touches."""
    lv = m_cap + 2
    ngrp = nt // g
    small = 6 * (nt // 64) * lv  # words: the wave-per-cell list (eight or four groups)
    big = 6 * lv                 # words: the workgroup-per-cell list (one group)
    alloc = max(big, small)
    for grp in range(ngrp):
        levels_end = grp * 5 * lv + 5 * lv
        coff_begin = ngrp * 5 * lv + grp * lv
        assert levels_end <= ngrp * 5 * lv <= coff_begin
        assert coff_begin + lv <= alloc, (nt, g, grp)
        # level indices 0 .. m_cap + 1 stay inside each array of lv entries
        assert m_cap + 1 < lv


@pytest.mark.parametrize("nt,g", [(256, 64), (256, 256), (512, 64), (512, 512)])
def test_lds_layout_of_reuse_groups(nt, g):
    for m_cap in (1, 2, 8, 64, 255):
        lds_check(nt, g, m_cap)


@pytest.mark.parametrize("sz", [4, 8])
def test_scratch_layout_fits_reservation(sz):
    for n in (2, 3, 255, 256, 511, 4097, 65536, 1 << 20):
        assert scratch_used(n, sz) <= scratch_bytes(n, sz), (n, sz)


def reuse_cases():
    """The benchmark's instances (every 64th of the 4096-instance batch, up to
    16384 particles) with the reusing adaptive depth, plus two that redo every
    step up to m_cap."""
    N, eps, alpha, init = W.batched_homogeneous(4096, seed=0)
    out = []
    for i in range(0, 4096, 64):
        if N[i] <= 16384:
            out.append((int(N[i]), float(eps[i]), float(alpha[i]), int(init[i]), i, {}))
    out.append((3000, 0.1, 0.0, 0, 9001, {"delta1": 1e-12, "delta2": 2e-12}))
    out.append((500, 0.05, 0.0, 1, 9002, {"m_init": 1, "delta1": 1e-12, "delta2": 2e-12}))
    return out


def test_attempt_offsets_within_allocations():
    recs = []
    with orc.AttemptLog() as log:
        for n, e, a, kind, uid, extra in reuse_cases():
            v = W.bkw(n, 0.6, 0, 1000 + uid) if kind == 0 else W.bimaxwellian(n, 0, 1000 + uid)
            kw = dict(eps=e, alpha=a, trunc=orc.ADAPTIVE_REUSE, m_init=2, m_cap=64, uid=uid, dt=0.05, weight=1.0 / n)
            kw.update(extra)
            o = orc.Instance(*v, **kw)
            o.run(4)
    recs = log.records
    assert len(recs) > 100
    redone = [r for r in recs if r["mprev"] > 0]
    assert len(redone) > 20  # kept attempts are exercised
    for r in recs:
        n, cap = r["n"], coll_cap(r["n"])
        P = n - r["N0"]
        R0 = r["R0prev"] + r["R0"]
        # tree indices (j, rA, rB) of this attempt's collisions
        assert r["ncoll"] <= cap, r
        # level outputs: each level's requests from offset sum of the shallower levels
        assert r["sum_R"] <= 2 * cap, r
        assert r["sum_R"] <= 2 * r["ncoll"], r
        # finals of all attempts by rank from 0: the last final is R0 - 1 < n
        assert R0 <= n, r
        # this attempt's leaves are read at ranks R0prev .. R0prev + R0 - 1
        assert r["R0prev"] + r["R0"] <= n, r
        # borrowed leaves take roles N0 - 1, N0 - 2, ...: ranks P .. R0 - 1 < n
        assert r["borrowed"] == max(0, R0 - P) and r["borrowed"] <= r["N0"], r
        # thermalized roles from leaf_end = N0 + min(R0, P) on
        assert r["n_th"] == max(0, P - R0), r
        # draw offsets of the levels (coff) stay 32-bit; levels below the LDS arrays' size
        assert r["coff_max"] < 2 ** 32, r
        assert r["me"] <= 64 and r["mprev"] <= r["m"] <= 64, r
        # every output of a collision is taken by a request or final: 2 ncoll = sum_R + finals
        assert 2 * r["ncoll"] == r["sum_R"] + r["R0"], r
