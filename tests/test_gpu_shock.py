"""GPU parity of the open slab of the stationary shock (Sec. 5.2) against the
oracle: reservoirs at both ends inject particles every step and particles that
fly past an end leave.

FP64: the particle count, the per-cell counts and every integer of the step
exact, positions and velocities within the parity tolerance, over 20 steps;
graph replay equals eager launches.  FP32: the slab holds the Mach-3 shock, with
the time-averaged far-field density and temperature at the Rankine-Hugoniot
states.  Arrays too small for the entering particles give TRMC_ENOSPC without
touching memory past them.
"""
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from test_gpu_parity import compare, oracle_of  # noqa: E402


@pytest.fixture(scope="module")
def trmc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible ROCm GPU"
    import paper_1009_2768_amd as T
    T.load()
    return T


def say(*a):
    print("[gpu-case]", *a, flush=True)


def _shock(T, nc, ppc, precision, uid, eps=0.1, seed=2, cap_factor=1.5):
    x, vx, vy, vz, w, up, down, cap = W.shock(nc, ppc, seed=seed, capacity_factor=cap_factor)
    inst = T.Instance(n_particles=cap, geometry=T.SLAB1D, n_cells=nc, length=1.0, dt=W.shock_dt(1.0, nc), eps=eps,
                      alpha=1.0, trunc=T.ADAPTIVE, m_init=2, m_cap=64, particle_weight=w, uid=uid, seed=seed,
                      precision=precision, bc=T.BC_INFLOW, n_live0=len(x), in_left=up, in_right=down)
    return inst, {"x": x, "vx": vx, "vy": vy, "vz": vz}, up, down


def test_open_slab_fp64_matches_oracle(trmc, orc):
    T = trmc
    inst, a, _, _ = _shock(T, 50, 100, T.FP64, uid=91)
    say(f"open slab fp64: 50 cells, {len(a['x'])} particles at start, capacity {inst.n_particles}, 20 steps")
    parts = [T.device_particles(a["vx"], a["vy"], a["vz"], a["x"], T.FP64, capacity=inst.n_particles)]
    ctx = T.Context([inst], parts)
    o = oracle_of(orc, inst, a)
    for s in range(20):
        ctx.step(1)
        o.run(1)
        assert ctx.count(0) == o.n, f"step {s}: gpu {ctx.count(0)} oracle {o.n}"
    got, mom = ctx.read(0), ctx.moments(0)
    ctx.close()
    compare(o, got, mom, 50)


def test_open_slab_graph_replay_equals_eager(trmc):
    T = trmc
    inst, a, _, _ = _shock(T, 40, 80, T.FP64, uid=92)
    say("open slab fp64: graph replay against eager, 10 steps")
    out = []
    for graph in (False, True):
        parts = [T.device_particles(a["vx"], a["vy"], a["vz"], a["x"], T.FP64, capacity=inst.n_particles)]
        ctx = T.Context([inst], parts)
        ctx.use_graph(graph)
        ctx.step(10)
        out.append((ctx.count(0), ctx.read(0)))
        ctx.close()
    assert out[0][0] == out[1][0]
    for k in ("x", "vx", "vy", "vz"):
        np.testing.assert_array_equal(out[0][1][k], out[1][1][k])


def test_fp32_holds_the_mach3_shock(trmc):
    T = trmc
    nc = 50
    inst, a, up, down = _shock(T, nc, 1000, T.FP32_MIXED, uid=93)
    say(f"open slab fp32: the paper's 50 cells x 1000 particles, {len(a['x'])} at start, 400 steps")
    parts = [T.device_particles(a["vx"], a["vy"], a["vz"], a["x"], T.FP32_MIXED, capacity=inst.n_particles)]
    ctx = T.Context([inst], parts)
    ctx.use_graph(True)
    rho, temp = [], []
    for s in range(400):
        ctx.step(1)
        if s >= 200 and s % 4 == 0:
            m = ctx.moments(0)
            rho.append(m["rho"])
            temp.append(m["T"])
    ctx.close()
    rho, temp = np.mean(rho, 0), np.mean(temp, 0)
    say(f"  upstream rho {rho[:5].mean():.3f} T {temp[:5].mean():.3f}; downstream rho {rho[-8:].mean():.3f} "
        f"T {temp[-8:].mean():.3f}")
    assert np.all(np.abs(rho[:5] - up[0]) < 0.03 * up[0]) and np.all(np.abs(temp[:5] - up[2]) < 0.03 * up[2])
    assert np.all(np.abs(rho[-8:] - down[0]) < 0.04 * down[0])
    assert np.all(np.abs(temp[-8:] - down[2]) < 0.04 * down[2])


def test_full_arrays_give_enospc(trmc):
    T = trmc
    x, vx, vy, vz, w, up, down, _ = W.shock(20, 50, seed=3)
    cap = len(x) + 8  # far fewer than one step's entries
    inst = T.Instance(n_particles=cap, geometry=T.SLAB1D, n_cells=20, length=1.0, dt=W.shock_dt(1.0, 20), eps=0.1,
                      alpha=1.0, trunc=T.ADAPTIVE, particle_weight=w, uid=94, precision=T.FP64, bc=T.BC_INFLOW,
                      n_live0=len(x), in_left=up, in_right=down)
    say("open slab with full arrays")
    parts = [T.device_particles(vx, vy, vz, x, T.FP64, capacity=cap)]
    ctx = T.Context([inst], parts)
    ctx.step(1)
    with pytest.raises(T.TrmcError) as e:
        ctx.count(0)
    assert e.value.code == -28
    ctx.close()


def test_open_slab_filling_from_empty_matches_oracle(trmc, orc):
    """No particle at admission: the reservoirs fill the slab; counts exact and
    states within the parity tolerance after 12 steps."""
    T = trmc
    up, down = W.shock_states()
    nc, w, cap = 20, 1.0 / 20 / 200, 60000
    e = np.zeros(0)
    inst = T.Instance(n_particles=cap, geometry=T.SLAB1D, n_cells=nc, length=1.0, dt=W.shock_dt(1.0, nc), eps=0.1,
                      alpha=1.0, trunc=T.ADAPTIVE, m_init=2, m_cap=64, particle_weight=w, uid=95, seed=4,
                      precision=T.FP64, bc=T.BC_INFLOW, n_live0=0, in_left=up, in_right=down)
    a = {"x": e, "vx": e, "vy": e, "vz": e}
    say("open slab fp64 filling from empty, 12 steps")
    parts = [T.device_particles(e, e, e, e, T.FP64, capacity=cap)]
    ctx = T.Context([inst], parts)
    o = oracle_of(orc, inst, a)
    for s in range(12):
        ctx.step(1)
        o.run(1)
        assert ctx.count(0) == o.n, f"step {s}"
    got, mom = ctx.read(0), ctx.moments(0)
    ctx.close()
    assert o.n > 0
    compare(o, got, mom, nc)
