"""GPU: the serving loop (continuous batching under an HBM budget).

A Poisson stream of homogeneous solves and shock tubes is served with a budget
that holds only a few requests at once, so requests wait, are admitted while
others run and retire at different ticks.  Every request completes, the budget
is never exceeded, and each captured result is bitwise the same as the same
request run alone in a fresh context (FP32-mixed and FP64).
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible ROCm GPU"
    import paper_1009_2768_amd as T
    T.load()
    return T


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def alone(T, req, precision):
    import torch
    from paper_1009_2768_amd.serve import instance_of
    inst = instance_of(req, precision)
    dt = torch.float32 if precision == T.FP32_MIXED else torch.float64
    parts = W.serving_initial(req, dtype=dt)
    ctx = T.Context([inst], [parts])
    ctx.step(int(req["steps"]))
    out = ctx.read(0)
    mom = ctx.moments(0)
    ctx.close()
    return out, mom


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_served_results_equal_alone(T, prec):
    from paper_1009_2768_amd.serve import Server, summarize
    precision = T.FP32_MIXED if prec == "fp32" else T.FP64
    reqs = W.serving_requests(rate=60.0, duration=0.25, seed=3, n_min=500, n_max=20000, steps_min=3,
                              steps_max=12, ppc_left=64)
    say(f"serving {len(reqs)} requests ({prec}), slabs {sum(r['slab'] for r in reqs)}")
    assert len(reqs) >= 8
    probe = [r["rid"] for r in reqs[:: max(1, len(reqs) // 5)]]
    srv = Server(hbm_budget=0, precision=precision, max_instances=64, max_cells=1 << 16, capture=probe)
    # a budget of about three average requests: requests must queue and join later
    costs = [srv.cost(r)[1] for r in reqs]
    srv.budget = int(max(max(costs), 3 * np.mean(costs)))
    done = srv.run(reqs, realtime=False)
    srv.close()
    assert sorted(d.rid for d in done) == [r["rid"] for r in reqs]
    assert srv.peak_bytes <= srv.budget
    assert srv.peak_active >= 2
    late = [d for d in done if d.tick_admitted > 0]
    assert late, "no request was admitted while others ran"
    st = summarize(done, srv.wall)
    say(f"p50 {st['p50_ms']:.1f} ms, p99 {st['p99_ms']:.1f} ms, {st['particle_steps_per_s']:.3e} ps/s")
    by = {d.rid: d for d in done}
    for rid in probe:
        req = next(r for r in reqs if r["rid"] == rid)
        ref, mom = alone(T, req, precision)
        got = by[rid].state
        for c in ("x", "vx", "vy", "vz"):
            if ref[c] is not None:
                assert np.array_equal(ref[c], got[c]), (rid, c)
        assert np.array_equal(np.asarray(mom["m_state"]), np.asarray(by[rid].moments["m_state"]))
        assert np.array_equal(np.asarray(mom["collisions"]), np.asarray(by[rid].moments["collisions"]))


def test_served_fp64_requests_match_oracle(T, orc):
    """Requests served in a mix (FP64) against the oracle run from the same
    initial particles (read back from the device recipe): integers of the last
    step exact, velocities within 1e-12 of the cell's thermal speed, positions
    within 1e-12 of the cell width."""
    import math

    import torch
    from paper_1009_2768_amd.serve import Server, instance_of
    reqs = W.serving_requests(rate=60.0, duration=0.3, seed=4, n_min=500, n_max=20000, steps_min=3,
                              steps_max=10, ppc_left=64)
    probe = [r["rid"] for r in reqs[:: max(1, len(reqs) // 6)]]
    say(f"serving {len(reqs)} requests (fp64) against the oracle, probes {probe}")
    srv = Server(hbm_budget=0, precision=T.FP64, max_instances=64, max_cells=1 << 16, capture=probe)
    costs = [srv.cost(r)[1] for r in reqs]
    srv.budget = int(max(max(costs), 3 * np.mean(costs)))
    done = srv.run(reqs, realtime=False)
    srv.close()
    by = {d.rid: d for d in done}
    kinds = set()
    for rid in probe:
        req = next(r for r in reqs if r["rid"] == rid)
        inst = instance_of(req, T.FP64)
        a = {k: (v.cpu().numpy() if v is not None else None)
             for k, v in W.serving_initial(req, dtype=torch.float64).items()}
        kw = dict(seed=inst.seed, uid=inst.uid, dt=inst.dt, eps=inst.eps, alpha=inst.alpha, trunc=inst.trunc,
                  m_init=inst.m_init, m_cap=inst.m_cap, delta1=inst.delta1, delta2=inst.delta2,
                  length=inst.length, weight=inst.particle_weight)
        if req["slab"]:
            kw.update(geometry=orc.SLAB, n_cells=inst.n_cells, x=a["x"])
        o = orc.Instance(a["vx"], a["vy"], a["vz"], **kw)
        o.run(int(req["steps"]))
        got, mom = by[rid].state, by[rid].moments
        nc = inst.n_cells if req["slab"] else 1
        kinds.add((req["slab"], inst.alpha))
        for c in range(nc):
            r = o.last[c]
            assert int(mom["collisions"][c]) == int(r.collisions), (rid, c)
            assert int(mom["thermalized"][c]) == int(r.n_th), (rid, c)
            assert int(mom["m_used"][c]) == int(r.m_used), (rid, c)
            assert int(mom["m_state"][c]) == int(o.m_state[c]), (rid, c)
        if req["slab"]:
            assert np.array_equal(np.asarray(mom["n"]), o.counts.astype(np.asarray(mom["n"]).dtype))
            err = float(np.abs(got["x"] - o.x[:o.n]).max() * nc)
            assert err <= 1e-12, (rid, "x", err)
        ov = np.stack([o.vx[:o.n], o.vy[:o.n], o.vz[:o.n]], 1)
        gv = np.stack([got["vx"], got["vy"], got["vz"]], 1)
        Tc = ov.var(0).sum() / 3.0
        err = float(np.abs(gv - ov).max() / math.sqrt(Tc))
        assert err <= 1e-12, (rid, "v", err)
    say(f"served requests matched the oracle: kinds (slab, alpha) {sorted(kinds)}")
    assert (True, 1.0) in kinds and any(not s for s, _ in kinds)


def test_request_larger_than_budget_is_rejected(T):
    from paper_1009_2768_amd.serve import Server
    reqs = W.serving_requests(rate=50.0, duration=0.1, seed=5, n_min=5000, n_max=6000, steps_min=2, steps_max=3)
    srv = Server(hbm_budget=1024, max_instances=8, max_cells=1 << 12)
    with pytest.raises(RuntimeError):
        srv.run(reqs, realtime=False)
    srv.close()


def test_admission_budget_behind_the_abi(T):
    """trmc_set_budget / TRMC_EBUSY: admissions beyond the device-memory budget of
    the active instances fail and change nothing; a retirement makes room."""
    from paper_1009_2768_amd import _abi
    from paper_1009_2768_amd.serve import Server, instance_of
    reqs = W.serving_requests(rate=100.0, duration=0.2, seed=6, n_min=2000, n_max=3000, steps_min=2,
                              steps_max=3, slab_fraction=0.0)
    assert len(reqs) >= 4
    srv = Server(hbm_budget=1 << 40, precision=T.FP32_MIXED, max_instances=8, max_cells=64)
    cost = [srv.cost(r)[1] for r in reqs[:4]]
    ctx = srv.ctx
    ctx.set_budget(cost[0] + cost[1])
    s0 = ctx.admit(instance_of(reqs[0]), W.serving_initial(reqs[0]))
    s1 = ctx.admit(instance_of(reqs[1]), W.serving_initial(reqs[1]))
    with pytest.raises(T.TrmcError) as e:
        ctx.admit(instance_of(reqs[2]), W.serving_initial(reqs[2]))
    assert e.value.code == _abi.EBUSY
    ctx.step(1)
    ctx.sync()
    ctx.retire(s0)
    if cost[2] <= cost[0]:
        s2 = ctx.admit(instance_of(reqs[2]), W.serving_initial(reqs[2]))
        ctx.step(1)
        ctx.sync()
        assert s2 != s1
    ctx.set_budget(0)  # no budget: anything that fits the slot table is admitted
    ctx.admit(instance_of(reqs[3]), W.serving_initial(reqs[3]))
    ctx.step(1)
    ctx.sync()
    srv.close()
