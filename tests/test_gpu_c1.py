"""GPU: the space-homogeneous BKW configuration as stated (Maxwell molecules,
N = 10^4, FP64, BKW initial data at K0 = 3/5, eps in {1, 0.1, 0.01}, dt = 0.05,
100 steps, seed 0), through the C ABI.

* Trajectory parity: after every one of the 100 steps the integers of the step
  (split, trees, leaves, thermalized count, depth, attempts) equal the oracle's
  and the velocities agree to 1e-12 of the thermal speed; natural (untruncated)
  and adaptive depth.
* BKW: an ensemble of 32 instances run together; the centred fourth moment
  follows the exact BKW decay, E[M4(t) - 15 T^2] = (M4(0) - 15 T^2) e^{-t/(3 eps)}
  (the untruncated Wild sum is the exact homogeneous solution over a step), and
  the ensemble mean of M4 at t = 5 matches the closed form 15 - 15 (1 - K0)^2
  e^{-t/(3 eps)} within 3 sigma; momentum and energy are conserved.
"""
import math
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

N, DT, STEPS, K0 = 10_000, 0.05, 100, 0.6
INT_FIELDS = [("N0", "N0"), ("m_eff", "m_eff"), ("R0", "R0"), ("thermalized", "n_th"), ("borrowed", "borrowed"),
              ("collisions", "collisions"), ("dummies", "dummies"), ("attempts", "attempts"),
              ("m_used", "m_used")]


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


@pytest.mark.parametrize("eps", [1.0, 0.1, 0.01])
@pytest.mark.parametrize("trunc", ["natural", "adaptive"])
def test_c1_every_step_matches_oracle(trmc, orc, eps, trunc):
    """The oracle runs its 100 steps on a host thread (its C code releases the
    interpreter lock) while the GPU runs and reads back every step."""
    import threading
    T = trmc
    say("C1 trajectory", eps, trunc)
    vx, vy, vz = W.bkw(N, K0, seed=0, stream=0)
    tr = T.NATURAL if trunc == "natural" else T.ADAPTIVE
    m_cap = 2048 if trunc == "natural" else 64
    o = orc.Instance(vx, vy, vz, eps=eps, alpha=0.0, trunc=orc.NATURAL if trunc == "natural" else orc.ADAPTIVE,
                     m_init=2, m_cap=m_cap, dt=DT, seed=0, uid=0, weight=1.0 / N)
    ref = []

    def oracle_steps():
        for _ in range(STEPS):
            o.run(1)
            r = o.last[0]
            ref.append(({ok: int(getattr(r, ok)) for _, ok in INT_FIELDS}, int(o.m_state[0]),
                        np.stack([o.vx, o.vy, o.vz], 1).copy()))

    th = threading.Thread(target=oracle_steps)
    th.start()
    inst = T.Instance(n_particles=N, eps=eps, alpha=0.0, trunc=tr, m_init=2, m_cap=m_cap, dt=DT, seed=0, uid=0,
                      precision=T.FP64, particle_weight=1.0 / N)
    ctx = T.Context([inst], [T.device_particles(vx, vy, vz, precision=T.FP64)])
    gpu = []
    try:
        for s in range(STEPS):
            ctx.step(1)
            got, mom = ctx.read(0), ctx.moments(0)
            gpu.append((mom, np.stack([got["vx"], got["vy"], got["vz"]], 1)))
    finally:
        ctx.close()
        th.join()
    assert len(ref) == STEPS
    worst = 0.0
    for s, ((ints, mstate, ov), (mom, gv)) in enumerate(zip(ref, gpu)):
        for gk, ok in INT_FIELDS:
            assert int(mom[gk][0]) == ints[ok], f"step {s}: {gk}"
        assert int(mom["m_state"][0]) == mstate, f"step {s}: m_state"
        assert int(mom["status"][0]) == 0
        Tc = ov.var(0).sum() / 3.0
        err = float(np.abs(gv - ov).max() / math.sqrt(Tc))
        worst = max(worst, err)
        assert err <= 1e-12, f"step {s}: max |dv|/sqrt(T) = {err:.3e}"
    say(f"C1 eps {eps} {trunc}: 100 steps, worst |dv|/sqrt(T) {worst:.2e}")


def centred(v):
    u = v.mean(1, keepdims=True)
    d = v - u
    e = (d * d).sum(0)
    return float(e.mean() / 3.0), float((e * e).mean())


@pytest.mark.parametrize("eps", [1.0, 0.1, 0.01])
def test_c1_bkw_fourth_moment(trmc, eps):
    T = trmc
    reps = 32
    say("C1 BKW ensemble", eps, reps)
    insts, parts, init = [], [], []
    for r in range(reps):
        vx, vy, vz = W.bkw(N, K0, seed=0, stream=100 + r)
        init.append(np.stack([vx, vy, vz]))
        insts.append(T.Instance(n_particles=N, eps=eps, alpha=0.0, trunc=T.NATURAL, m_init=2, m_cap=2048, dt=DT,
                                seed=0, uid=r, precision=T.FP64, particle_weight=1.0 / N))
        parts.append(T.device_particles(vx, vy, vz, precision=T.FP64))
    ctx = T.Context(insts, parts)
    ctx.step(STEPS)
    out = [ctx.read(k) for k in range(reps)]
    ctx.close()
    decay = math.exp(-STEPS * DT / (3.0 * eps))
    d, m4 = [], []
    for r in range(reps):
        v0 = init[r]
        v1 = np.stack([out[r]["vx"], out[r]["vy"], out[r]["vz"]])
        T0, M0 = centred(v0)
        T1, M1 = centred(v1)
        # exact conservation of momentum and energy (FP64 rounding)
        assert np.allclose(v1.sum(1), v0.sum(1), rtol=0, atol=1e-9 * np.abs(v0).sum())
        assert (v1 * v1).sum() == pytest.approx((v0 * v0).sum(), rel=1e-12)
        d.append((M1 - 15 * T1 * T1) - (M0 - 15 * T0 * T0) * decay)
        m4.append(M1 / (T1 * T1))
    d, m4 = np.array(d), np.array(m4)
    sd = d.std(ddof=1) / math.sqrt(reps)
    assert abs(d.mean()) <= 3.0 * sd, (d.mean(), sd)
    closed = 15.0 - 15.0 * (1.0 - K0) ** 2 * decay  # per unit temperature
    sdm = m4.std(ddof=1) / math.sqrt(reps)
    # the initial ensemble's own spread around the closed form at t = 0 adds to the noise
    assert abs(m4.mean() - closed) <= 3.0 * math.hypot(sdm, 0.27 * decay / math.sqrt(reps)), (m4.mean(), closed)
    say(f"C1 BKW eps {eps}: M4/T^2 {m4.mean():.4f} +- {sdm:.4f}, closed form {closed:.4f}")
