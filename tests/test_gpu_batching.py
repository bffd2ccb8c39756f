"""GPU: batching — schedules and the captured step.

A batch of uneven instances (homogeneous cells of very different sizes, Maxwell
and hard spheres, slabs) is stepped under each kernel path of the schedule and
with the step replayed from a captured HIP graph.  The schedule only changes how
the cells are mapped onto the GPU: every integer of the step (split, trees,
thermalized count, depth) must agree exactly and the FP64 velocities and
positions to 1e-12 relative (the cell sums are reduced in a different order).  Graph replay runs
the same kernels with the same arguments, so it must agree bitwise with eager
launches, replay after replay, with eager work and synchronisations in between
and after the work tables change (admission, retirement).
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

INT_KEYS = ("N0", "R0", "thermalized", "collisions", "m_eff", "m_used", "attempts", "borrowed", "m_state")


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


def batch(T, prec):
    """Uneven mix: homogeneous cells from 3 to 40000 particles, both kernels, and a slab."""
    insts, arrays = [], []
    spec = [(3, 0.5, 0.0), (64, 0.1, 1.0), (700, 0.02, 0.0), (2500, 1.0, 1.0), (9000, 0.05, 0.0),
            (40000, 0.2, 1.0), (300, 5.0, 0.0), (17000, 1e-3, 1.0)]
    for k, (n, eps, alpha) in enumerate(spec):
        vx, vy, vz = W.bimaxwellian(n, stream=50 + k) if k % 2 else W.bkw(n, 0.6, stream=50 + k)
        insts.append(T.Instance(n_particles=n, eps=eps, alpha=alpha, trunc=T.ADAPTIVE, m_cap=64, uid=10 + k,
                                precision=prec))
        arrays.append({"vx": vx, "vy": vy, "vz": vz})
    x, vx, vy, vz, w = W.sod(40, 60, 20, seed=0, stream=77)
    insts.append(T.Instance(n_particles=len(x), geometry=T.SLAB1D, n_cells=40, eps=0.01, alpha=1.0,
                            dt=W.sod_dt(1.0, 40), particle_weight=w, trunc=T.ADAPTIVE, m_cap=64, uid=99,
                            precision=prec))
    arrays.append({"x": x, "vx": vx, "vy": vy, "vz": vz})
    return insts, arrays


def make_ctx(T, insts, arrays):
    parts = [T.device_particles(a["vx"], a["vy"], a["vz"], a.get("x"), i.precision) for i, a in zip(insts, arrays)]
    return T.Context(insts, parts)


def snapshot(ctx, n):
    return [(ctx.read(k), ctx.moments(k)) for k in range(n)]


@pytest.mark.parametrize("path", ["group", "wave", "tiled"])
def test_schedule_does_not_change_results(trmc, path):
    T = trmc
    say("schedule invariance, path", path)
    insts, arrays = batch(T, T.FP64)
    ref = make_ctx(T, insts, arrays)  # library default schedule
    alt = make_ctx(T, insts, arrays)
    code = {"group": T.PATH_GROUP, "wave": T.PATH_WAVE, "tiled": T.PATH_TILED}[path]
    alt.set_schedule([code] * T.SCHED_BUCKETS)
    assert alt.get_schedule() == [code] * T.SCHED_BUCKETS
    for step in range(3):
        ref.step(1)
        alt.step(1)
        for k, ((ra, rm), (aa, am)) in enumerate(zip(snapshot(ref, len(insts)), snapshot(alt, len(insts)))):
            for key in INT_KEYS:
                assert np.array_equal(np.asarray(rm[key]), np.asarray(am[key])), (step, k, key)
            # positions follow the velocities of the previous step: same tolerance
            for c in ("x", "vx", "vy", "vz"):
                a, b = ra[c], aa[c]
                if a is None:
                    continue
                scale = max(1.0, float(np.abs(a).max()))
                assert np.abs(a - b).max() <= 1e-12 * scale, (step, k, c)
    ref.close()
    alt.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_replay_matches_eager(trmc, prec):
    import torch
    T = trmc
    p = T.FP64 if prec == "fp64" else T.FP32_MIXED
    say("graph replay vs eager", prec)
    insts, arrays = batch(T, p)
    eager = make_ctx(T, insts, arrays)
    graph = make_ctx(T, insts, arrays)
    graph.use_graph(True)
    junk = torch.zeros(1 << 16, device="cuda")
    for step in range(4):
        eager.step(1)
        graph.step(1)
        junk.add_(1.0)  # unrelated eager work between replays
        torch.cuda.synchronize()
        for k, ((ra, rm), (ga, gm)) in enumerate(zip(snapshot(eager, len(insts)), snapshot(graph, len(insts)))):
            for c in ("x", "vx", "vy", "vz"):
                if ra[c] is not None:
                    assert np.array_equal(ra[c], ga[c]), (step, k, c)
            for key in INT_KEYS:
                assert np.array_equal(np.asarray(rm[key]), np.asarray(gm[key])), (step, k, key)
    # several steps per call, then a change of the tables (retire + admit): re-capture
    eager.step(3)
    graph.step(3)
    eager.retire(2)
    graph.retire(2)
    n = 5000
    vx, vy, vz = W.bkw(n, 0.6, stream=123)
    extra = T.Instance(n_particles=n, eps=0.3, alpha=0.0, trunc=T.ADAPTIVE, m_cap=64, uid=500, precision=p)
    se = eager.admit(extra, T.device_particles(vx, vy, vz, None, p))
    sg = graph.admit(extra, T.device_particles(vx, vy, vz, None, p))
    assert se == sg
    eager.step(2)
    graph.step(2)
    for k in [0, 1, 3, se]:
        ra, ga = eager.read(k), graph.read(k)
        for c in ("vx", "vy", "vz"):
            assert np.array_equal(ra[c], ga[c]), (k, c)
    graph.use_graph(False)
    eager.step(1)
    graph.step(1)
    assert np.array_equal(eager.read(se)["vx"], graph.read(se)["vx"])
    eager.close()
    graph.close()


def test_autotuner_table_is_valid(trmc):
    T = trmc
    from paper_1009_2768_amd.autotune import autotune
    say("autotuner")
    insts, arrays = batch(T, T.FP32_MIXED)
    parts = [T.device_particles(a["vx"], a["vy"], a["vz"], a.get("x"), i.precision) for i, a in zip(insts, arrays)]
    before = [p["vx"].clone() for p in parts]
    table, timings = autotune(insts, parts, warmup=1, steps=1)
    assert len(table) == T.SCHED_BUCKETS
    for b, res in timings.items():
        best = min(res, key=res.get)
        assert all(t > 0 for t in res.values())
        assert table[b] == best or (table[b] == T.PATH_GROUP and res[best] > 0.95 * res[T.PATH_GROUP])
    for p, b in zip(parts, before):  # the tuner steps copies only
        assert torch_equal(p["vx"], b)
    ctx = T.Context(insts, parts)
    ctx.set_schedule(table)
    ctx.step(2)
    ctx.sync()
    ctx.close()


def test_mix_refinement_keeps_paths_valid(trmc):
    """The refinement on the whole mix only picks, for a bucket, a path its cells
    can take, steps copies only, and a table it returns runs the batch."""
    T = trmc
    from paper_1009_2768_amd.autotune import candidates, refine_for_mix
    say("mix refinement")
    insts, arrays = batch(T, T.FP32_MIXED)
    parts = [T.device_particles(a["vx"], a["vy"], a["vz"], a.get("x"), i.precision) for i, a in zip(insts, arrays)]
    before = [p["vx"].clone() for p in parts]
    start = [T.PATH_GROUP] * T.SCHED_BUCKETS
    table = refine_for_mix(insts, parts, start, warmup=1, steps=1)
    assert len(table) == T.SCHED_BUCKETS
    for b in range(T.SCHED_BUCKETS):
        mine = [i for i in insts if T.size_bucket(i) == b]
        if not mine:
            assert table[b] == start[b]
        else:
            assert table[b] in candidates(mine), (b, table[b])
    for p, b in zip(parts, before):
        assert torch_equal(p["vx"], b)
    ctx = T.Context(insts, parts)
    ctx.set_schedule(table)
    ctx.step(2)
    ctx.sync()
    ctx.close()


def torch_equal(a, b):
    import torch
    return bool(torch.equal(a, b))
