"""GPU: cells whose previous step thermalized every particle make their role
permutation (a6) only when an attempt keeps or collides a particle, and take
the removed set's and the normals' sums from the moments pass when the attempt
does thermalize every particle.  At an eps where the split (Alg. 4.2) leaves a
cell sometimes wholly thermalized and sometimes not, and, for contrast, at ones
where it keeps about half (sometimes more, sometimes less) or more than half of
the particles (borrowed leaves, redos), every step's integers equal the FP64
oracle's, the velocities stay within 1e-12 of it, and fused steps equal single
steps bitwise; on the workgroup, the wave and the tile path, with fixed and
adaptive depth."""
import math
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


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


# Maxwell molecules (g = 1, rho = 1): q = exp(-dt / eps).  "thermal": q = 1 / (f n),
# f chosen so that about half the steps (adaptive: with redos) thermalize the
# whole cell.  "kept": q n = n/2 - 1/2, so that half the steps keep half the
# particles (N0 = n/2) and half do not (N0 = n/2 - 1).  "kept60": q = 0.6, every
# step keeps more than half (adaptive: with borrowed leaves and redos).
CASES = {"group": 2000, "wave": 300, "tiled": 20000}
FACTOR = {"fixed": 16.0, "adaptive": 100.0}


def eps_of(kind, trunc, n):
    if kind == "thermal":
        return 0.05 / math.log(FACTOR[trunc] * n)
    q = (n / 2 - 0.5) / n if kind == "kept" else 0.6
    return -0.05 / math.log(q)


@pytest.mark.parametrize("kind", ["thermal", "kept", "kept60"])
@pytest.mark.parametrize("path", ["group", "wave", "tiled"])
@pytest.mark.parametrize("trunc", ["fixed", "adaptive"])
def test_roles_when_needed_match_oracle(trmc, orc, kind, path, trunc):
    T = trmc
    n, steps = CASES[path], 40
    eps = eps_of(kind, trunc, n)
    say("roles when needed", kind, path, trunc, "n", n, "eps", f"{eps:.4g}")
    v = W.bkw(n, 0.6, 0, 321)
    tr, otr = (T.FIXED, orc.FIXED) if trunc == "fixed" else (T.ADAPTIVE, orc.ADAPTIVE)
    mk = lambda: T.Instance(n_particles=n, eps=eps, alpha=0.0, trunc=tr, m_init=2, m_cap=64, uid=5, seed=11,
                            dt=0.05, precision=T.FP64, particle_weight=1.0 / n)
    p = {"group": T.PATH_GROUP, "wave": T.PATH_WAVE, "tiled": T.PATH_TILED}[path]
    o = orc.Instance(*v, eps=eps, alpha=0.0, trunc=otr, m_init=2, m_cap=64, uid=5, seed=11, dt=0.05,
                     weight=1.0 / n)
    ctx = T.Context([mk()], [T.device_particles(*v, precision=T.FP64)])
    ctx.set_schedule([p] * T.SCHED_BUCKETS)
    whole = 0
    for s in range(steps):
        ctx.step(1)
        o.run(1)
        mom, r = ctx.moments(0), o.last[0]
        for gk, ok in (("N0", "N0"), ("R0", "R0"), ("thermalized", "n_th"), ("collisions", "collisions"),
                       ("dummies", "dummies"), ("attempts", "attempts"), ("m_used", "m_used")):
            assert int(mom[gk][0]) == int(getattr(r, ok)), (s, gk, int(mom[gk][0]), int(getattr(r, ok)))
        whole += (int(r.n_th) == n) if kind == "thermal" else (2 * int(r.N0) >= n)
    single = ctx.read(0)
    ctx.close()
    say(f"{whole} of {steps} steps " + ("thermalized the whole cell" if kind == "thermal" else "kept half or more"))
    if kind == "kept60":
        assert whole == steps, whole
    else:
        assert 5 <= whole <= steps - 5, whole  # both kinds of step, and the changes between them
    ov = np.stack([o.vx, o.vy, o.vz], 1)
    gv = np.stack([single["vx"], single["vy"], single["vz"]], 1)
    err = float(np.abs(gv - ov).max() / math.sqrt(ov.var(0).sum() / 3.0))
    assert err <= 1e-12, err
    ctx = T.Context([mk()], [T.device_particles(*v, precision=T.FP64)])
    ctx.set_schedule([p] * T.SCHED_BUCKETS)
    ctx.step(steps)
    fused = ctx.read(0)
    ctx.close()
    for c in ("vx", "vy", "vz"):
        assert np.array_equal(fused[c], single[c]), c


@pytest.mark.parametrize("sched", ["default", "tiled"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_restart_through_the_shortcuts_is_bitwise(trmc, prec, sched):
    """A run restarted from its saved state (step index, adaptive depths) equals
    the uninterrupted run bitwise, also where the step's shortcuts apply (roles
    made only when needed, the whole cell's sums from the moments pass, the
    normals summed early, the majorant from its bracket), which a restarted
    context takes from a blank record."""
    T = trmc
    P = T.FP64 if prec == "fp64" else T.FP32_MIXED
    say("restart through the shortcuts", prec, sched)
    specs = [(3000, 1e-4, 0.0), (2000, 0.05 / math.log(100.0 * 2000), 0.0), (6000, 0.01, 1.0), (300, 1e-4, 1.0),
             (4000, 0.2, 1.0)]
    insts, arrs = [], []
    for k, (n, eps, alpha) in enumerate(specs):
        v = W.bkw(n, 0.6, 0, 500 + k) if k % 2 == 0 else W.bimaxwellian(n, 0, 500 + k)
        insts.append(dict(n_particles=n, eps=eps, alpha=alpha, trunc=T.ADAPTIVE, m_init=2, m_cap=64, uid=60 + k,
                          seed=9, dt=0.05, precision=P, particle_weight=1.0 / n))
        arrs.append(v)

    def ctx_of(kw_list, arr_list):
        ctx = T.Context([T.Instance(**kw) for kw in kw_list],
                        [T.device_particles(*a, precision=P) for a in arr_list])
        if sched == "tiled":
            ctx.set_schedule([T.PATH_TILED] * T.SCHED_BUCKETS)
        return ctx

    ctx = ctx_of(insts, arrs)
    ctx.step(8)
    full = [ctx.read(k) for k in range(len(insts))]
    ctx.close()
    ctx = ctx_of(insts, arrs)
    ctx.step(4)
    mid = [ctx.read(k) for k in range(len(insts))]
    ctx.close()
    again = [dict(kw, step0=4, m_state0=m["m_state"]) for kw, m in zip(insts, mid)]
    ctx = ctx_of(again, [(m["vx"], m["vy"], m["vz"]) for m in mid])
    ctx.step(4)
    out = [ctx.read(k) for k in range(len(insts))]
    ctx.close()
    for k in range(len(insts)):
        for c in ("vx", "vy", "vz"):
            assert np.array_equal(full[k][c], out[k][c]), (k, c)


@pytest.mark.parametrize("path", ["group", "wave", "tiled"])
def test_restarted_before_every_step_is_bitwise(trmc, orc, path):
    """A run restarted before every step (a blank record: no cell is predicted
    wholly thermalized, roles are made up front) equals the uninterrupted run bit
    for bit, on every path, at an eps where predictions fail.  On the tile path a
    cell predicted wholly thermalized whose first attempt is wholly thermalized
    but whose redo keeps or collides particles makes its roles and block sums
    inside the collision kernel, in the order of the tile kernels; the oracle's
    attempt log shows that the run has such steps."""
    T = trmc
    n, steps = {"group": 2000, "wave": 300, "tiled": 20000}[path], 12
    eps = 0.05 / math.log(100.0 * n)
    v = W.bkw(n, 0.6, 0, 321)
    kw = dict(n_particles=n, eps=eps, alpha=0.0, trunc=T.ADAPTIVE, m_init=2, m_cap=64, uid=5, seed=11, dt=0.05,
              precision=T.FP64, particle_weight=1.0 / n)
    say("restarted before every step", path, n, f"{eps:.4g}")
    o = orc.Instance(*v, eps=eps, alpha=0.0, trunc=orc.ADAPTIVE, m_init=2, m_cap=64, uid=5, seed=11, dt=0.05,
                     weight=1.0 / n)
    fallback, failed, prev = 0, 0, False
    for s_ in range(steps):
        with orc.AttemptLog() as log:
            o.run(1)
        first = log.records[0]["n_th"] == n
        last = int(o.last[0].n_th) == n
        fallback += int(prev and first and not last)
        failed += int(prev and not last)
        prev = last
    say(f"failed predictions: {failed}, of which after a wholly thermalized first attempt: {fallback}")
    assert failed >= 1
    if path == "tiled":
        assert fallback >= 1

    tiled = [{"group": T.PATH_GROUP, "wave": T.PATH_WAVE, "tiled": T.PATH_TILED}[path]] * T.SCHED_BUCKETS
    ctx = T.Context([T.Instance(**kw)], [T.device_particles(*v, precision=T.FP64)])
    ctx.set_schedule(tiled)
    ctx.step(steps)
    full = ctx.read(0)
    ctx.close()
    cur, m_state = v, None
    for s_ in range(steps):
        ctx = T.Context([T.Instance(**dict(kw, step0=s_, m_state0=m_state))],
                        [T.device_particles(*cur, precision=T.FP64)])
        ctx.set_schedule(tiled)
        ctx.step(1)
        r = ctx.read(0)
        ctx.close()
        cur, m_state = (r["vx"], r["vy"], r["vz"]), r["m_state"]
    for k, c in enumerate(("vx", "vy", "vz")):
        assert np.array_equal(full[c], cur[k]), c
