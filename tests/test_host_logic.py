"""CPU checks of the host-side logic: schedule buckets, autotuner candidates,
serving request streams and descriptors, the stored-counter guard of the
benchmark.  No GPU call is made."""
import math
import os
import sys

import numpy as np
import pytest
from scipy import stats

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


@pytest.fixture(scope="module")
def T():
    import paper_1009_2768_amd as T
    return T


def test_size_bucket_is_floor_log2_of_particles_per_cell(T):
    for n in [1, 2, 3, 255, 256, 257, 65535, 65536, 10**6, 2**31]:
        inst = T.Instance(n_particles=n)
        assert T.size_bucket(inst) == int(math.floor(math.log2(n)))
    slab = T.Instance(n_particles=12000, geometry=T.SLAB1D, n_cells=40)
    assert T.size_bucket(slab) == int(math.floor(math.log2(12000 / 40)))


def test_autotune_candidates_follow_the_path_rules(T):
    from paper_1009_2768_amd.autotune import candidates
    homog = [T.Instance(n_particles=5000, m_cap=64)]
    slab = [T.Instance(n_particles=5000, geometry=T.SLAB1D, n_cells=10, m_cap=64)]
    deep = [T.Instance(n_particles=5000, m_cap=2048)]
    assert candidates(homog) == [T.PATH_GROUP, T.PATH_WAVE, T.PATH_TILED]
    assert candidates(slab) == [T.PATH_GROUP, T.PATH_WAVE]  # no tile path for slab cells
    assert candidates(deep) == [T.PATH_GROUP]  # wave and tile paths need m_cap <= 256


def test_serving_stream_is_poisson_with_the_stated_ranges():
    reqs = W.serving_requests(rate=200.0, duration=20.0, seed=1)
    t = np.array([r["arrival"] for r in reqs])
    assert np.all(np.diff(t) > 0) and t[-1] < 20.0
    # exponential gaps of mean 1/200 (Kolmogorov-Smirnov)
    assert stats.kstest(np.diff(t), "expon", args=(0, 1 / 200.0)).pvalue > 1e-3
    assert abs(len(reqs) - 4000) < 5 * math.sqrt(4000)
    homog = [r for r in reqs if not r["slab"]]
    n = np.array([r["n"] for r in homog])
    assert n.min() >= 1000 and n.max() <= 10**6
    # log-uniform sizes: log N uniform on [log 1e3, log 1e6]
    u = (np.log(n) - math.log(1e3)) / (math.log(1e6) - math.log(1e3))
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    steps = np.array([r["steps"] for r in reqs])
    assert steps.min() >= 50 and steps.max() <= 500
    eps = np.array([r["eps"] for r in reqs])
    assert eps.min() >= 1e-4 and eps.max() <= 1.0
    frac = np.mean([r["slab"] for r in reqs])
    assert abs(frac - 0.5) < 5 * math.sqrt(0.25 / len(reqs))
    for r in reqs:
        if r["slab"]:
            nc, left = r["n_cells"], r["n_cells"] // 2
            assert 2 <= nc <= 12288 and nc % 2 == 0
            assert (r["ppc_left"], r["ppc_right"]) == (888, 111) and r["alpha"] == 1.0
            assert r["n"] == left * r["ppc_left"] + (nc - left) * r["ppc_right"]
    # homogeneous solves: Maxwell molecules and hard spheres 50/50, BKW and bi-Maxwellian 50/50
    hard = np.mean([r["alpha"] == 1.0 for r in homog])
    assert abs(hard - 0.5) < 5 * math.sqrt(0.25 / len(homog))
    bkw = np.mean([r["init"] == 0 for r in homog])
    assert abs(bkw - 0.5) < 5 * math.sqrt(0.25 / len(homog))
    # tubes of 888 / 111 particles per cell: n_cells = N / 499.5 up to rounding to an even count
    for r in reqs:
        if r["slab"] and r["n_cells"] > 2:
            assert abs(r["n"] - r["n_cells"] * 499.5) <= 1.0


def test_serving_initial_data_moments():
    """Homogeneous serving requests start from BKW (K = 3/5: M4 = 12.6, T = 1) or
    the bi-Maxwellian (P_xx = 2, T = 4/3); the draws are the device recipe, run on
    the CPU here."""
    import torch
    n = 400_000
    for init, m4, pxx in ((0, 12.6, 1.0), (1, None, 2.0)):
        req = {"rid": 7 + init, "seed": 3, "slab": False, "n": n, "init": init}
        p = W.serving_initial(req, device="cpu", dtype=torch.float64)
        v = np.stack([p["vx"].numpy(), p["vy"].numpy(), p["vz"].numpy()])
        e2 = (v * v).sum(0)
        assert abs(v.mean(1)).max() < 5 * math.sqrt(2.0 / n)
        assert abs((v[0] ** 2).mean() - pxx) < 5 * math.sqrt(8.0 / n)
        if m4 is not None:
            # E|v|^4 = 12.6; its variance for BKW at K = 0.6 is below 2000
            assert abs(e2.var() + e2.mean() ** 2 - m4) < 5 * math.sqrt(2000.0 / n)
            assert abs(e2.mean() - 3.0) < 5 * math.sqrt(20.0 / n)


def test_serving_descriptors(T):
    from paper_1009_2768_amd.serve import instance_of
    reqs = W.serving_requests(rate=50.0, duration=1.0, seed=2)
    for r in reqs:
        inst = instance_of(r)
        assert inst.uid == r["rid"] and inst.n_particles == r["n"] and inst.trunc == T.ADAPTIVE
        if r["slab"]:
            dx = 1.0 / r["n_cells"]
            assert inst.geometry == T.SLAB1D and inst.n_cells == r["n_cells"]
            assert math.isclose(inst.dt, 0.5 * dx / 3.0) and math.isclose(inst.particle_weight, dx / r["ppc_left"])
            assert inst.alpha == 1.0
        else:
            assert inst.geometry == T.HOMOG and math.isclose(inst.particle_weight, 1.0 / r["n"])
            assert inst.alpha == r["alpha"] and r["alpha"] in (0.0, 1.0)


def test_batched_workload_parameters():
    N, eps, alpha, init = W.batched_homogeneous(4096, seed=0)
    assert N.min() >= 256 and N.max() <= 65536 and int(N.sum()) == 48356870
    assert eps.min() >= 1e-4 and eps.max() <= 10.0
    assert np.array_equal(alpha, np.arange(4096) % 2)
    assert set(np.unique(init)) == {0, 1}


def test_stored_traffic_needs_matching_sources(tmp_path, monkeypatch):
    import json

    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "k_collide_batched_homogeneous_4096.traffic.json")))
    assert rec["bytes_per_launch"] > 0
    # the stored figure is reported only for the kernel sources it was measured on
    monkeypatch.setattr(bench, "source_sha256", lambda: "0" * 64)
    assert bench.stored_traffic("k_collide<float>", None) is None


def test_unpack_moments_reads_the_abi_records(T):
    """The records trmc_moments_async writes (trmc_cell_moments, as laid out in
    the header) decode into the same dict as Context.moments."""
    import ctypes

    from paper_1009_2768_amd import _abi
    nc = 3
    recs = (_abi.CellMoments * nc)()
    for c in range(nc):
        recs[c].n = 100 + c
        recs[c].m_state = 2 * c + 1
        recs[c].rho = 0.5 * c
        recs[c].M4 = 15.0 + c
        recs[c].collisions = (1 << 40) + c
        recs[c].wb_thermalized = 7 * c
        recs[c].q = 1.0 / (c + 2)
    raw = np.frombuffer(bytes(recs), dtype=np.uint8)
    assert T.moments_record_bytes(nc) == len(raw) == nc * ctypes.sizeof(_abi.CellMoments)
    got = T.unpack_moments(np.concatenate([raw, np.zeros(40, np.uint8)]), nc)  # longer buffer: first nc
    assert sorted(got) == sorted(f[0] for f in _abi.CellMoments._fields_)
    for c in range(nc):
        for name, _ in _abi.CellMoments._fields_:
            assert got[name][c] == getattr(recs[c], name), (c, name)
