"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's
formula: they compare with published known-answer values, library routines,
closed forms derived from the Wild sum, brute-force enumeration, or invariants.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import special, stats

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------------------------
# Random numbers: Philox4x32-10
# ----------------------------------------------------------------------------
def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(t, 16) for t in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers(orc):
    """Published known-answer vectors of Philox4x32-10 (Salmon et al., SC'11)."""
    for ctr, key, expect in _kat():
        assert orc.philox(ctr, key).tolist() == expect


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_library(orc, tmp_path):
    """Cross-check against rocRAND's Philox4x32-10 engine, called as a library."""
    exe = tmp_path / "rocrand_check"
    subprocess.check_call(["hipcc", "-O1", "-o", str(exe), os.path.join(HERE, "rocrand_philox_check.cpp")])
    g = np.random.default_rng(1)
    lines, expect = [], []
    for _ in range(200):
        c = [int(g.integers(0, 2**32)), int(g.integers(0, 2**29)), int(g.integers(0, 2**32)),
             int(g.integers(0, 2**32))]
        k = [int(g.integers(0, 2**32)), int(g.integers(0, 2**32))]
        lines.append(" ".join("%x" % w for w in c + k))
        expect.append(orc.philox(c, k).tolist())
    out = subprocess.run([str(exe)], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         check=True).stdout.split("\n")
    got = [[int(t, 16) for t in ln.split()] for ln in out if ln.strip()]
    assert got == expect


# ----------------------------------------------------------------------------
# exp(-x), the majorant grid, the keyed permutation
# ----------------------------------------------------------------------------
def test_exp_neg_within_one_ulp_of_libm(orc):
    g = np.random.default_rng(2)
    xs = np.concatenate([g.random(20000) * 745.0, g.random(20000) * 5.0, 10.0 ** g.uniform(-12, 0, 5000),
                         np.arange(0, 700, 0.25)])
    for x in xs:
        e = orc.exp_neg(float(x))
        r = math.exp(-float(x))
        assert abs(e - r) <= math.ulp(r), (x, e, r)
    assert orc.exp_neg(0.0) == 1.0
    assert orc.exp_neg(800.0) == 0.0


def test_grid_up_is_smallest_20_bit_majorant(orc):
    g = np.random.default_rng(3)
    for x in np.concatenate([g.random(2000) * 20, 10.0 ** g.uniform(-5, 5, 2000), [1.0, 2.0, 0.75]]):
        y = orc.grid_up(float(x))
        assert y >= x
        m, e = math.frexp(y)
        assert (m * 2**20) == int(m * 2**20)  # at most 20 significant bits
        assert y - x < 2.0 ** (e - 20) * 1.0000001  # less than one grid step above
        assert orc.grid_up(y) == y


@pytest.mark.parametrize("n", [2, 3, 5, 7, 16, 17, 100, 255, 256, 257, 1000, 4097])
def test_perm_is_bijection(orc, n):
    keys = orc.philox([n, 2 << 24, 0, 0], [0, 0])
    img = [orc.perm(i, n, keys) for i in range(n)]
    assert sorted(img) == list(range(n))


@pytest.mark.parametrize("n", [2, 3, 6, 11, 17])
def test_perm_positions_uniform(orc, n):
    """Each element is equally likely at each position over keys (chi-square)."""
    trials = 6000
    counts = np.zeros((n, n))
    for t in range(trials):
        keys = orc.philox([t, 2 << 24, n, 0], [1, 2])
        for i in range(n):
            counts[i, orc.perm(i, n, keys)] += 1
    chi2 = ((counts - trials / n) ** 2 / (trials / n)).sum()
    assert chi2 < stats.chi2.ppf(0.9995, (n - 1) ** 2)


@pytest.mark.parametrize("n", [300, 1000, 4097, 70000])
def test_perm_positions_uniform_in_bins(orc, n):
    """Larger domains (odd and even bit counts, heavy cycle walking at 4097):
    element bins against position bins over keys are uniform (chi-square), and
    the position of an element is uncorrelated with its index."""
    trials, nb = 400, 8
    rng = np.random.default_rng(n)
    idx = rng.choice(n, size=64, replace=False)
    counts = np.zeros((nb, nb))
    corr = []
    for t in range(trials):
        keys = orc.philox([t, 2 << 24, n, 7], [3, 4])
        pos = np.array([orc.perm(int(i), n, keys) for i in idx])
        counts[(idx * nb) // n, (pos * nb) // n] += 1
        corr.append(np.corrcoef(idx, pos)[0, 1])
    expect = counts.sum(1, keepdims=True) / nb
    chi2 = ((counts - expect) ** 2 / expect).sum()
    assert chi2 < stats.chi2.ppf(0.9995, nb * (nb - 1))
    # the mean correlation over keys of 64 pairs has standard deviation about 1/sqrt(63 * trials)
    assert abs(np.mean(corr)) < 5.0 / math.sqrt(63 * trials)


def test_perm_kept_set_is_uniform_over_slots(orc):
    """The unchanged set (the first N0 roles) covers every slot with frequency N0/n."""
    n, n0, trials = 50, 20, 3000
    hits = np.zeros(n)
    for t in range(trials):
        keys = orc.philox([t, 2 << 24, 5, 9], [1, 1])
        for r in range(n0):
            hits[orc.perm(r, n, keys)] += 1
    p = n0 / n
    z = (hits - trials * p) / math.sqrt(trials * p * (1 - p))
    assert np.abs(z).max() < 4.5


# ----------------------------------------------------------------------------
# Alg. 4.2: split into collision sets; eq. (WST-r) coefficients
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("tau,m", [(0.3, 2), (0.7, 5), (0.95, 64), (0.5, 1)])
def test_split_means_are_wild_sum_coefficients(orc, tau, m):
    """E[N_k] = N (1-tau) tau^k, E[N_{m+1}] = N tau^{m+1} (eq. WST-r, Alg. 4.2)."""
    n, trials = 1000, 4000
    q = 1.0 - tau
    acc = np.zeros(m + 2)
    acc2 = np.zeros(m + 2)
    for s in range(trials):
        N, me = orc.split(0, 5, 3, s, n, q, m)
        assert int(N.sum()) == n
        acc += N
        acc2 += N.astype(float) ** 2
    mean = acc / trials
    sd = np.sqrt(np.maximum(acc2 / trials - mean**2, 1e-12) / trials)
    expect = np.array([n * q * tau**k for k in range(m + 1)] + [n * tau ** (m + 1)])
    assert np.all(np.abs(mean - expect) <= 4.5 * sd + 1e-9), (mean, expect, sd)


def _split_law_bruteforce(n, q, m):
    """Exact law of (N_0..N_{m+1}) by enumerating the Iround outcomes."""
    law = {}

    def rec(k, rem, prefix, p):
        if (k > 0 and rem == 0) or k > m:
            key = tuple(prefix + [0] * (m + 1 - len(prefix)) + [rem])
            law[key] = law.get(key, 0.0) + p
            return
        y = q * rem
        f = math.floor(y)
        for val, pv in ((f, 1 - (y - f)), (f + 1, y - f)):
            if pv > 0 and val <= rem:
                rec(k + 1, rem - val, prefix + [val], p * pv)

    rec(0, n, [], 1.0)
    return law


@pytest.mark.parametrize("n,q,m", [(2, 0.4, 2), (3, 0.55, 3), (4, 0.3, 2), (4, 0.8, 4)])
def test_split_exact_law_small_n(orc, n, q, m):
    """Brute force of Alg. 4.2 for N <= 4 vs the oracle's frequencies (chi-square)."""
    law = _split_law_bruteforce(n, q, m)
    trials = 20000
    freq = {}
    for s in range(trials):
        N, me = orc.split(1, 2, 0, s, n, q, m)
        key = tuple(int(v) for v in N)
        freq[key] = freq.get(key, 0) + 1
    assert set(freq) <= set(law)
    chi2 = sum((freq.get(k, 0) - trials * p) ** 2 / (trials * p) for k, p in law.items() if p > 0)
    assert chi2 < stats.chi2.ppf(0.9995, max(1, len(law) - 1))


# ----------------------------------------------------------------------------
# Collision law: eq. (Maxwell_coll-r), eq. (n3d-r), Alg. 4.4
# ----------------------------------------------------------------------------
def test_pair_collision_conserves_and_keeps_relative_speed(orc):
    g = np.random.default_rng(4)
    for _ in range(2000):
        a, b = g.standard_normal(3) * 2, g.standard_normal(3)
        oa, ob, acc = orc.collide(a, b, g.random(), g.random())
        assert acc
        np.testing.assert_allclose(oa + ob, a + b, rtol=0, atol=1e-13)
        assert abs((oa @ oa + ob @ ob) - (a @ a + b @ b)) <= 1e-12 * (a @ a + b @ b)
        assert abs(np.linalg.norm(oa - ob) - np.linalg.norm(a - b)) <= 1e-12 * np.linalg.norm(a - b)


def test_direction_matches_paper_arccos_parametrisation(orc):
    """cos(theta) = 2 xi1 - 1 gives the same sigma as theta = arccos(2 xi1 - 1) (eq. n3d-r)."""
    g = np.random.default_rng(5)
    for _ in range(500):
        xi1, xi2 = g.random(), g.random()
        a, b = np.array([1.0, 0.0, 0.0]), np.array([-1.0, 0.0, 0.0])
        oa, ob, _ = orc.collide(a, b, xi1, xi2)
        th, ph = math.acos(2 * xi1 - 1), 2 * math.pi * xi2
        sig = np.array([math.cos(ph) * math.sin(th), math.sin(ph) * math.sin(th), math.cos(th)])
        np.testing.assert_allclose(oa, sig * 1.0, atol=1e-12)  # c = 0, |q|/2 = 1
        np.testing.assert_allclose(ob, -sig, atol=1e-12)


def test_post_collision_direction_uniform_on_sphere(orc):
    g = np.random.default_rng(6)
    s = []
    for _ in range(20000):
        oa, ob, _ = orc.collide([0, 0, 0.5], [0, 0, -0.5], g.random(), g.random())
        s.append(oa / 0.5)
    s = np.array(s)
    np.testing.assert_allclose(s.mean(axis=0), 0, atol=4 / math.sqrt(3 * 20000) * 1.2)
    np.testing.assert_allclose(s.T @ s / len(s), np.eye(3) / 3, atol=0.012)
    # each component of a uniform unit vector is uniform on [-1, 1] (Archimedes)
    assert stats.kstest(s[:, 2], "uniform", args=(-1, 2)).pvalue > 1e-3
    assert stats.kstest(s[:, 0], "uniform", args=(-1, 2)).pvalue > 1e-3


def test_vhs_dummy_collision_acceptance(orc):
    """Alg. 4.4: accepted iff Sigma xi < sigma_ij, i.e. with probability |q|^alpha / g."""
    g = np.random.default_rng(7)
    a, b = np.array([0.3, 0.0, 0.0]), np.array([-0.2, 0.1, 0.0])
    qn = np.linalg.norm(a - b)
    for alpha, gmax in ((1.0, 2.0), (0.5, 1.5)):
        acc = 0
        for _ in range(20000):
            oa, ob, ok = orc.collide(a, b, g.random(), g.random(), g.random(), alpha, gmax)
            if not ok:
                assert np.array_equal(oa, a) and np.array_equal(ob, b)
            acc += ok
        p = qn**alpha / gmax
        assert abs(acc / 20000 - p) < 4.5 * math.sqrt(p * (1 - p) / 20000)


# ----------------------------------------------------------------------------
# Transport and the stable sort (splitting of Sec. 3.1)
# ----------------------------------------------------------------------------
def test_transport_matches_unfolded_reflection(orc):
    """Specular walls: the reflected position is the free position folded into [0, L]."""
    g = np.random.default_rng(8)
    L = 1.0
    for _ in range(5000):
        x, v, dt = g.random() * L, g.standard_normal() * 5, g.random() * 0.7
        xn, vn, c = orc.transport(x, v, dt, L, 200)
        free = x + v * dt
        y = free % (2 * L)
        expect = y if y <= L else 2 * L - y
        flips = math.floor(free / L) if free >= 0 else -math.floor(free / L)
        assert abs(xn - expect) < 1e-12
        assert vn == (v if flips % 2 == 0 else -v) or abs(xn) < 1e-12 or abs(xn - L) < 1e-12
        assert c == min(199, int(math.floor(xn * 200 / L)))


def test_slab_sort_is_stable_counting_sort(orc):
    """Collisionless slab: the step reduces to transport + sort, which must equal numpy's
    stable argsort of the cell ids (a library routine)."""
    x, vx, vy, vz, w = W.sod(40, 60, 8, seed=3)
    g = np.random.default_rng(9)
    perm = g.permutation(len(x))  # scramble the input order
    x, vx, vy, vz = x[perm], vx[perm], vy[perm], vz[perm]
    inst = orc.Instance(vx, vy, vz, x=x, geometry=orc.SLAB, n_cells=40, dt=0.004, eps=1e300, weight=w)
    inst.run(1)
    xs, vxs = x.copy(), vx.copy()
    cells = np.array([0] * len(xs))
    for i in range(len(xs)):
        xs[i], vxs[i], cells[i] = orc.transport(xs[i], vxs[i], 0.004, 1.0, 40)
    order = np.argsort(cells, kind="stable")
    np.testing.assert_array_equal(inst.x, xs[order])
    np.testing.assert_array_equal(inst.vx, vxs[order])
    np.testing.assert_array_equal(inst.vy, vy[order])
    np.testing.assert_array_equal(inst.counts, np.bincount(cells, minlength=40))


def test_moments_match_numpy(orc):
    vx, vy, vz = W.bimaxwellian(5000, seed=1)
    inst = orc.Instance(vx, vy, vz)
    m = inst.moments()[0]
    v = np.stack([vx, vy, vz], 1)
    u = v.mean(0)
    np.testing.assert_allclose(m[1:4], u, atol=1e-14)
    np.testing.assert_allclose(m[5:8], v.var(0), rtol=1e-12)
    np.testing.assert_allclose(m[4], v.var(0).sum() / 3, rtol=1e-12)
    np.testing.assert_allclose(m[8], ((v**2).sum(1) ** 2).mean(), rtol=1e-12)
    assert m[0] == pytest.approx(1.0)
