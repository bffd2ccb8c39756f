"""GPU: fused steps.

A space-homogeneous cell's step reads nothing but the cell's own previous step,
so step(n) of a context whose instances are all homogeneous takes every cell
through its n steps inside one launch per collision kernel.  A fused step draws
with the same keys (instance, cell, step index) as a single step, so the
velocities, every per-cell counter, the adaptive depths and the step index must
agree bitwise with n single steps: for each kernel path and variant (workgroup
and wave per cell, tree-shape truncation, adaptive depth with reuse, cells too
small to collide), in FP32 and FP64, launched directly or replayed from the
captured graph.  A context holding a slab or a cell on the tiled path is not
fused and must agree as well.
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

INT_KEYS = ("n", "N0", "R0", "thermalized", "wb_thermalized", "collisions", "work_collisions", "dummies",
            "violations", "m_eff", "m_used", "attempts", "borrowed", "m_state", "status")
REAL_KEYS = ("q", "g", "rho", "ux", "uy", "uz", "T", "Pxx", "Pyy", "Pzz", "M4")


@pytest.fixture(scope="module")
def trmc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible ROCm GPU"
    import paper_1009_2768_amd as T
    T.load()
    return T


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def homogeneous_mix(T, prec):
    """Every whole-cell variant: group and wave cells, FIXED and ADAPTIVE depth,
    Maxwell and hard spheres, tree-shape truncation, reuse, a 1-particle cell."""
    spec = [
        # n, eps, alpha, trunc, extra
        (40000, 0.2, 1.0, T.ADAPTIVE, {}),
        (17000, 1e-3, 0.0, T.ADAPTIVE, {}),
        (9000, 0.05, 1.0, T.FIXED, {"m_init": 12}),
        (2500, 1.0, 0.0, T.ADAPTIVE, {}),
        (700, 0.02, 1.0, T.ADAPTIVE, {}),
        (300, 5.0, 0.0, T.FIXED, {"m_init": 6}),
        (64, 0.1, 1.0, T.ADAPTIVE, {}),
        (1, 0.5, 0.0, T.ADAPTIVE, {}),
        (6000, 0.2, 1.0, T.FIXED, {"m_init": 16, "wb": T.WB_MEAN, "wb_mmax": 3}),
        (5000, 0.05, 0.0, T.FIXED, {"m_init": 16, "wb": T.WB_MIN, "wb_mmax": 2}),
        (20000, 0.3, 1.0, T.ADAPTIVE_REUSE, {"m_init": 2, "delta1": 1e-6, "delta2": 2e-4}),
        (500, 0.05, 0.0, T.ADAPTIVE_REUSE, {"m_init": 1}),
        # every E_1 above delta2: the first step redoes up to m_cap
        (8000, 0.1, 1.0, T.ADAPTIVE, {"m_init": 2, "delta1": 1e-12, "delta2": 2e-12}),
        (3000, 0.1, 0.0, T.ADAPTIVE_REUSE, {"m_init": 2, "delta1": 1e-12, "delta2": 2e-12}),
    ]
    insts, arrays = [], []
    for k, (n, eps, alpha, trunc, extra) in enumerate(spec):
        vx, vy, vz = W.bimaxwellian(n, stream=300 + k) if k % 2 else W.bkw(n, 0.6, stream=300 + k)
        insts.append(T.Instance(n_particles=n, eps=eps, alpha=alpha, trunc=trunc, m_cap=64, uid=40 + k,
                                precision=prec, **extra))
        arrays.append({"vx": vx, "vy": vy, "vz": vz})
    return insts, arrays


def whole_cell_schedule(T):
    # wave per cell below 2^11 particles, workgroup per cell above: no tiled cell
    return [T.PATH_WAVE if b < 11 else T.PATH_GROUP for b in range(T.SCHED_BUCKETS)]


def make_ctx(T, insts, arrays, schedule=None):
    parts = [T.device_particles(a["vx"], a["vy"], a["vz"], a.get("x"), i.precision) for i, a in zip(insts, arrays)]
    ctx = T.Context(insts, parts)
    if schedule is not None:
        ctx.set_schedule(schedule)
    return ctx


def assert_same(T, a, b, n_inst, tag):
    for k in range(n_inst):
        ra, rb = a.read(k), b.read(k)
        assert ra["step"] == rb["step"], (tag, k)
        assert np.array_equal(ra["m_state"], rb["m_state"]), (tag, k)
        for c in ("x", "vx", "vy", "vz"):
            if ra[c] is not None:
                assert np.array_equal(ra[c], rb[c]), (tag, k, c)
        ma, mb = a.moments(k), b.moments(k)
        for key in INT_KEYS:
            assert np.array_equal(np.asarray(ma[key]), np.asarray(mb[key])), (tag, k, key)
        for key in REAL_KEYS:
            assert np.array_equal(np.asarray(ma[key]), np.asarray(mb[key])), (tag, k, key)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_fused_steps_equal_single_steps(trmc, prec):
    T = trmc
    p = T.FP64 if prec == "fp64" else T.FP32_MIXED
    say("fused vs single steps", prec)
    insts, arrays = homogeneous_mix(T, p)
    sched = whole_cell_schedule(T)
    fused = make_ctx(T, insts, arrays, sched)
    single = make_ctx(T, insts, arrays, sched)
    single.fuse_steps(False)
    fused.step(5)
    attempts = []
    for _ in range(5):
        single.step(1)
        attempts.append(max(int(single.moments(k)["attempts"].max()) for k in range(len(insts))))
    assert_same(T, fused, single, len(insts), "5 steps")
    # the counters really moved on, and some cell redid or extended an attempt
    assert fused.read(0)["step"] == 5
    assert max(attempts) > 1
    # a second fused call continues from the step index the first left; a call
    # longer than one launch's 32 steps is cut into launches
    fused.step(3)
    single.step(2)
    single.step(1)
    assert_same(T, fused, single, len(insts), "8 steps")
    fused.step(40)
    for _ in range(40):
        single.step(1)
    assert_same(T, fused, single, len(insts), "48 steps")
    assert fused.read(0)["step"] == 48
    fused.close()
    single.close()


def test_fused_steps_equal_graph_replay(trmc):
    T = trmc
    say("fused vs graph replay")
    insts, arrays = homogeneous_mix(T, T.FP32_MIXED)
    sched = whole_cell_schedule(T)
    fused = make_ctx(T, insts, arrays, sched)
    graph = make_ctx(T, insts, arrays, sched)
    graph.fuse_steps(False)
    graph.use_graph(True)
    fused.step(4)
    graph.step(4)
    assert_same(T, fused, graph, len(insts), "graph")
    # admission and retirement between fused calls
    fused.retire(3)
    graph.retire(3)
    n = 3000
    vx, vy, vz = W.bkw(n, 0.6, stream=321)
    extra = T.Instance(n_particles=n, eps=0.3, alpha=1.0, trunc=T.ADAPTIVE, m_cap=64, uid=700,
                       precision=T.FP32_MIXED)
    sf = fused.admit(extra, T.device_particles(vx, vy, vz, None, T.FP32_MIXED))
    sg = graph.admit(extra, T.device_particles(vx, vy, vz, None, T.FP32_MIXED))
    assert sf == sg
    fused.step(3)
    graph.step(3)
    for k in [0, 1, 2, 4, 10, sf]:
        ra, rg = fused.read(k), graph.read(k)
        assert ra["step"] == rg["step"]
        for c in ("vx", "vy", "vz"):
            assert np.array_equal(ra[c], rg[c]), (k, c)
    fused.close()
    graph.close()


@pytest.mark.parametrize("what", ["slab", "tiled"])
def test_unfusable_contexts_agree(trmc, what):
    """A slab (transport and sort between steps) or a cell on the tiled path
    keeps the step-by-step launches; the fuse switch must not change results."""
    T = trmc
    say("unfusable context", what)
    insts, arrays = homogeneous_mix(T, T.FP64)
    insts, arrays = insts[:4], arrays[:4]
    sched = whole_cell_schedule(T)
    if what == "slab":
        x, vx, vy, vz, w = W.sod(30, 50, 20, seed=0, stream=78)
        insts.append(T.Instance(n_particles=len(x), geometry=T.SLAB1D, n_cells=30, eps=0.01, alpha=1.0,
                                dt=W.sod_dt(1.0, 30), particle_weight=w, trunc=T.ADAPTIVE, m_cap=64, uid=98,
                                precision=T.FP64))
        arrays.append({"x": x, "vx": vx, "vy": vy, "vz": vz})
    else:
        sched[15] = T.PATH_TILED  # the 40000-particle cell
    a = make_ctx(T, insts, arrays, sched)
    b = make_ctx(T, insts, arrays, sched)
    b.fuse_steps(False)
    a.step(3)
    for _ in range(3):
        b.step(1)
    assert_same(T, a, b, len(insts), what)
    a.close()
    b.close()
