"""Benchmark: batched homogeneous TRMC-R, FP32 collisions with FP64 cell sums.

Workload (one GPU): 4096 independent space-homogeneous instances run together,
N per instance log-uniform in [256, 65536] (about 4.8e7 particles in total), eps
log-uniform in [1e-4, 10], Maxwell molecules and hard spheres alternating, BKW
or bi-Maxwellian initial data, dt = 0.05, adaptive depth (m_init 2, m_cap 64,
delta1 0.005, delta2 0.01).  A step is one collision step of every instance; the
metric is particle-steps per second over the timed steps (state resident in HBM).
By default 20 untimed steps come first: over them the adaptive depths settle (the
first steps redo many attempts) and the launch order learns each cell's cost, so
the 20 timed steps are the solver's steady regime.

The headline (value, roofline) is measured first.  Then, by default, the legs
cpu (the oracle on host threads), batching (batched against one instance at a
time), serving (a Poisson request stream, and the same requests all queued at
once) and precision (FP32 against FP64 per cell moment on the 10^7-particle
transition tube over 500 steps); --legs adds fusion, reuse, shock, tubes and wb.  A watchdog prints the
line after --budget seconds with the legs not reached listed as skipped.

Prints one JSON line.  --gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_batch(n_inst: int, seed: int, scale: float = 1.0):
    import numpy as np

    import workloads as W
    N, eps, alpha, init = W.batched_homogeneous(n_inst, seed=seed)
    if scale != 1.0:
        N = np.maximum(2, (N * scale).astype(np.int64))
    return N, eps, alpha, init


def build_context(T, N, eps, alpha, init, seed, precision, device="cuda", uids=None, trunc=None):
    import numpy as np
    import torch

    import workloads as W
    dt = torch.float32 if precision == T.FP32_MIXED else torch.float64
    total = int(N.sum())
    offs = np.concatenate([[0], np.cumsum(N)])
    vx = torch.empty(total, dtype=dt, device=device)
    vy = torch.empty(total, dtype=dt, device=device)
    vz = torch.empty(total, dtype=dt, device=device)
    insts, parts = [], []
    uids = list(range(len(N))) if uids is None else [int(u) for u in uids]
    for i in range(len(N)):
        n, uid = int(N[i]), uids[i]
        a = W.bkw(n, 0.6, seed, 1000 + uid) if init[i] == 0 else W.bimaxwellian(n, seed, 1000 + uid)
        sl = slice(int(offs[i]), int(offs[i + 1]))
        vx[sl].copy_(torch.from_numpy(a[0]))
        vy[sl].copy_(torch.from_numpy(a[1]))
        vz[sl].copy_(torch.from_numpy(a[2]))
        insts.append(T.Instance(n_particles=n, eps=float(eps[i]), alpha=float(alpha[i]), dt=0.05,
                                trunc=T.ADAPTIVE if trunc is None else trunc, m_init=2, m_cap=64,
                                precision=precision, uid=uid, seed=seed))
        parts.append({"vx": vx[sl], "vy": vy[sl], "vz": vz[sl], "x": None})
    ctx = T.Context(insts, parts)
    return ctx, (vx, vy, vz)


# the sources the timed collision kernel is compiled from
KERNEL_SOURCES = ("k_collide.hip", "collide_core.h", "trmc_device.h", "trmc_internal.h")


def source_sha256() -> str:
    """Hash of the collision kernel's sources (names and contents), to tell whether
    stored HBM counter figures still describe the kernel being timed."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_1009_2768_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_collide_batched_homogeneous_4096.traffic.json")


def stored_traffic(kernel: str, table, steps_per_launch: int = 1):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's counters), or None when the
    kernel sources differ from those the counters were taken with, or the counters
    were taken on launches of another number of steps.  The caller asks only when
    the step is that one kernel (no cell on the tile path)."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != source_sha256() or kernel not in rec.get("kernel", ""):
        return None
    if int(rec.get("steps_per_launch", 1)) != steps_per_launch:
        return None
    return rec["bytes_per_launch"]


def traffic_record(kernel: str):
    """The committed counter record itself (bytes per launch, steps per launch,
    schedule) while the kernel sources match it, else None: reported beside a
    run of another number of steps per launch, whose own launch was not counted."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != source_sha256() or kernel not in rec.get("kernel", ""):
        return None
    return {"bytes_per_launch": rec["bytes_per_launch"], "steps_per_launch": rec.get("steps_per_launch", 1),
            "schedule": rec.get("table")}


def time_steps(ctx, steps, warmup, fuse):
    """`warmup` untimed steps, then exactly `steps` timed steps on the context's
    stream, synchronised on both sides.  fuse: one call for all the timed steps
    (each homogeneous cell goes through them in one launch, results identical to
    single steps); else one call per step, replayed from the captured graph.
    Returns the wall time of the timed steps (s) and the HIP-event time per step
    (ms) measured on the library's stream."""
    import numpy as np
    import torch
    ctx.fuse_steps(fuse)
    stream = ctx.stream
    if fuse:
        ctx.step(warmup)
    else:
        for _ in range(warmup):
            ctx.step(1)
    ctx.sync()
    torch.cuda.synchronize()
    if fuse:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            e0.record(stream)
            ctx.step(steps)
            e1.record(stream)
        ctx.sync()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall, e0.elapsed_time(e1) / steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for k in range(steps):
            ev[k][0].record(stream)
            ctx.step(1)
            ev[k][1].record(stream)
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, float(np.mean([a.elapsed_time(b) for a, b in ev]))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores(cap: int = 16) -> int:
    """Host cores this process may use, at most `cap` (a GPU machine shares its host
    between GPUs: 16 cores per GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def cpu_baseline(N, eps, alpha, init, seed, budget_s=15.0, stride=16):
    """The FP64 oracle on a bounded sample of the same batch: every stride-th
    instance, spread over host threads (the oracle is C called through ctypes,
    which releases the interpreter lock, and its instances share nothing).  Each
    thread steps its instances round after round until the time budget is spent;
    the rate is all particle-steps done over the wall time."""
    import threading

    import oracle
    import workloads as W
    idx = list(range(0, len(N), stride))
    insts = []
    for i in idx:
        n = int(N[i])
        a = W.bkw(n, 0.6, seed, 1000 + i) if init[i] == 0 else W.bimaxwellian(n, seed, 1000 + i)
        insts.append(oracle.Instance(a[0], a[1], a[2], eps=float(eps[i]), alpha=float(alpha[i]), dt=0.05,
                                     trunc=oracle.ADAPTIVE, m_init=2, m_cap=64, uid=i, seed=seed,
                                     weight=1.0 / n))
    oracle.lib()
    cores = host_cores()
    # deal the instances to threads largest first, each to the least loaded thread
    shares = [[] for _ in range(cores)]
    load = [0] * cores
    for k in sorted(range(len(insts)), key=lambda k: -insts[k].n):
        t = load.index(min(load))
        shares[t].append(insts[k])
        load[t] += insts[k].n
    done = [0] * cores
    steps = [0] * cores
    t_end = time.perf_counter() + budget_s

    def work(t):
        while time.perf_counter() < t_end:
            for inst in shares[t]:
                inst.run(1)
                done[t] += inst.n
            steps[t] += 1

    t0 = time.perf_counter()
    th = [threading.Thread(target=work, args=(t,)) for t in range(cores) if shares[t]]
    for x in th:
        x.start()
    for x in th:
        x.join()
    wall = time.perf_counter() - t0
    return {"value": sum(done) / wall, "unit": "particle-steps/s", "cores": len(th), "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{len(insts)} instances (every {stride}th of the batch, {sum(i.n for i in insts)} "
                      f"particles), {min(steps)}-{max(steps)} steps each, serial FP64 oracle per instance on "
                      f"{len(th)} host threads, {wall:.1f} s"}


def batching_speedup(T, N, eps, alpha, init, seed, prec, table, stride=16, steps=3):
    """Batched versus one instance at a time on the same sample (every stride-th
    instance): each instance alone in its own context (the plain one-instance
    path, a graph per step), then all of them in one context; same schedule,
    same steps, results identical (per-instance keys)."""
    import numpy as np
    import torch
    idx = np.arange(0, len(N), stride)
    Ns, es, al, ini = N[idx], eps[idx], alpha[idx], init[idx]
    ctx, bufs = build_context(T, Ns, es, al, ini, seed, prec, uids=idx)
    ctx.set_schedule(table)
    ctx.use_graph(True)
    ctx.step(1)
    ctx.sync()
    t0 = time.perf_counter()
    ctx.step(steps)
    ctx.sync()
    batched = (time.perf_counter() - t0) / steps
    ctx.close()
    alone = 0.0
    for k in range(len(idx)):
        c1, _ = build_context(T, Ns[k:k + 1], es[k:k + 1], al[k:k + 1], ini[k:k + 1], seed, prec, uids=idx[k:k + 1])
        c1.set_schedule(table)
        c1.use_graph(True)
        c1.step(1)
        c1.sync()
        t0 = time.perf_counter()
        c1.step(steps)
        c1.sync()
        alone += (time.perf_counter() - t0) / steps
        c1.close()
    torch.cuda.synchronize()
    return {"instances": int(len(idx)), "particles": int(Ns.sum()), "one_at_a_time_ms_per_step": alone * 1e3,
            "batched_ms_per_step": batched * 1e3, "speedup": alone / batched}


def work_totals(T, ctx):
    """Collisions of the accepted results and over all adaptive attempts, and the
    cells that redid their step, in the last step of every instance."""
    coll = work = redo = 0
    for k in range(len(ctx.instances)):
        m = ctx.moments(k)
        coll += int(m["collisions"].sum())
        work += int(m["work_collisions"].sum())
        redo += int((m["attempts"] > 1).sum())
    return {"collisions": coll, "work_collisions": work, "cells_redone": redo}


def adaptive_reuse(T, N, eps, alpha, init, seed, prec, table, steps, warmup, fuse):
    """The benchmark workload with the adaptive depth that keeps rejected attempts
    (Sec. 4.3, the collisions of the wrong depth reused) instead of recomputing
    them: same instances, schedule and timing."""
    import torch
    ctx, bufs = build_context(T, N, eps, alpha, init, seed, prec, trunc=T.ADAPTIVE_REUSE)
    ctx.set_schedule(table)
    ctx.use_graph(True)
    wall, kernel_ms = time_steps(ctx, steps, warmup, fuse)
    out = {"ms_per_step": wall * 1e3 / steps, "kernel_ms": kernel_ms,
           "particle_steps_per_s": int(N.sum()) * steps / wall}
    out.update(work_totals(T, ctx))
    ctx.close()
    del ctx, bufs
    torch.cuda.empty_cache()
    return out


def step_fusion(T, N, eps, alpha, init, seed, prec, table, steps, warmup, fused_ms):
    """The timed steps again, on a twin context (same inputs, same warmup, so the
    same steps), one launch per step replayed from the captured graph instead of
    one launch for all of them."""
    import torch
    ctx, bufs = build_context(T, N, eps, alpha, init, seed, prec)
    ctx.set_schedule(table)
    ctx.use_graph(True)
    ctx.fuse_steps(False)
    for _ in range(warmup):
        ctx.step(1)
    wall, kernel_ms = time_steps(ctx, steps, 0, False)
    ctx.close()
    del ctx, bufs
    torch.cuda.empty_cache()
    return {"fused_ms_per_step": fused_ms, "unfused_ms_per_step": wall * 1e3 / steps,
            "unfused_kernel_ms": kernel_ms, "speedup": wall * 1e3 / steps / fused_ms}


def tree_shape_truncation(T, n_inst, seed, steps=5):
    """Tree-shape truncation (Sec. 4.4) beside the plain step on one workload:
    n_inst homogeneous hard-sphere instances of 50,000 bi-Maxwellian particles
    (the paper's homogeneous test size), eps = 0.2, fixed depth 24, FP32 with
    FP64 sums.  Plain, def:2 with m_max 2 and def:3 with m_max 3, same keys, all
    on the workgroup-per-cell path (the only path of the truncated step)."""
    import numpy as np
    import torch

    import workloads as W
    n = 50_000
    out = {"workload": f"{n_inst} homogeneous hard-sphere instances x {n} particles, bi-Maxwellian, eps 0.2, "
                       "dt 0.05, fixed depth 24, fp32", "particles": n_inst * n}
    for name, wb, mmax in (("plain", T.WB_OFF, 1), ("def2_mmax2", T.WB_MIN, 2), ("def3_mmax3", T.WB_MEAN, 3)):
        insts, parts = [], []
        for i in range(n_inst):
            a = W.bimaxwellian(n, seed, 5000 + i)
            insts.append(T.Instance(n_particles=n, eps=0.2, alpha=1.0, dt=0.05, trunc=T.FIXED, m_init=24, m_cap=64,
                                    precision=T.FP32_MIXED, uid=5000 + i, seed=seed, wb=wb, wb_mmax=mmax))
            parts.append({k: torch.from_numpy(v.astype(np.float32)).cuda() for k, v in zip(("vx", "vy", "vz"), a)})
        ctx = T.Context(insts, parts)
        ctx.set_schedule([T.PATH_GROUP] * T.SCHED_BUCKETS)
        ctx.use_graph(True)
        ctx.step(1)
        ctx.sync()
        t0 = time.perf_counter()
        ctx.step(steps)
        ctx.sync()
        dt = (time.perf_counter() - t0) / steps
        mom = [ctx.moments(k) for k in range(n_inst)]
        th = sum(int(m["thermalized"][0]) for m in mom)
        wbt = sum(int(m["wb_thermalized"][0]) for m in mom)
        coll = sum(int(m["collisions"][0]) for m in mom)
        out[name] = {"ms_per_step": dt * 1e3, "particle_steps_per_s": n_inst * n / dt,
                     "thermalized_fraction": th / (n_inst * n), "tree_shape_fraction": wbt / (n_inst * n),
                     "collisions_per_particle": coll / (n_inst * n)}
        ctx.close()
        del ctx, parts
        torch.cuda.empty_cache()
        log(f"tree-shape truncation {name}: {out[name]}")
    return out


def stationary_shock(T, seed, steps=400, average_from=200):
    """The paper's stationary shock (Sec. 5.2): Mach 3, 50 cells, 1000 upstream
    particles per cell, reservoirs at both ends, hard spheres, adaptive depth, FP32.
    For eps 1, 0.1 and 1e-3: time per step (graph replay), and the time-averaged
    far-field density and temperature against the Rankine-Hugoniot states."""
    import numpy as np
    import torch

    import workloads as W
    nc = 50
    x, vx, vy, vz, w, up, down, cap = W.shock(nc, 1000, seed=seed)
    out = {"workload": "Mach-3 stationary shock, 50 cells x 1000 upstream particles per cell, reservoirs at both "
                       "ends, hard spheres, adaptive depth, fp32", "steps": steps,
           "rankine_hugoniot": {"rho": [up[0], down[0]], "T": [up[2], down[2]]}}
    for eps in (1.0, 0.1, 1e-3):
        inst = T.Instance(n_particles=cap, geometry=T.SLAB1D, n_cells=nc, length=1.0, dt=W.shock_dt(1.0, nc),
                          eps=eps, alpha=1.0, trunc=T.ADAPTIVE, m_init=2, m_cap=64, particle_weight=w, uid=7000,
                          seed=seed, precision=T.FP32_MIXED, bc=T.BC_INFLOW, n_live0=len(x), in_left=up,
                          in_right=down)
        parts = [T.device_particles(vx, vy, vz, x, T.FP32_MIXED, capacity=cap)]
        ctx = T.Context([inst], parts)
        ctx.use_graph(True)
        ctx.step(average_from)
        ctx.sync()
        rho, temp, ps, wall = [], [], 0, 0.0
        for s in range(steps - average_from):
            n0 = ctx.count(0)
            t0 = time.perf_counter()
            ctx.step(1)
            ctx.sync()
            wall += time.perf_counter() - t0
            ps += n0
            if s % 4 == 0:
                m = ctx.moments(0)
                rho.append(m["rho"])
                temp.append(m["T"])
        ctx.close()
        rho, temp = np.mean(rho, 0), np.mean(temp, 0)
        out[f"eps_{eps:g}"] = {"ms_per_step": wall * 1e3 / (steps - average_from), "particle_steps_per_s": ps / wall,
                               "rho_up": float(rho[:5].mean()), "rho_down": float(rho[-8:].mean()),
                               "T_up": float(temp[:5].mean()), "T_down": float(temp[-8:].mean())}
        log(f"stationary shock eps {eps:g}: {out[f'eps_{eps:g}']}")
        del parts
        torch.cuda.empty_cache()
    return out


def tubes(T, seed, steps=20, warmup=5):
    """The two shock-tube workloads in FP32 with FP64 cell sums, hard spheres,
    adaptive depth, specular walls, dt = CFL 0.5: the Sod tube (200 cells, 500
    particles per cell on average, eps 1e-2) and the transition-regime tube
    (10^4 cells x 1000 particles on average, eps(x) log-linear from 1e-4 to 1).
    A slab's steps are not fused (transport and sort between steps): one graph
    replay per step, timed with HIP events on the library's stream."""
    import torch

    import workloads as W
    out = {}
    for name, nc, ppl, ppr, eps in (("sod_200", 200, 889, 111, 1e-2),
                                    ("transition_1e4", 10000, 1778, 222, None)):
        x, vx, vy, vz, w = W.sod(nc, ppl, ppr, seed=seed)
        e = W.transition_eps(nc) if eps is None else None
        inst = T.Instance(n_particles=len(x), geometry=T.SLAB1D, n_cells=nc, dt=W.sod_dt(1.0, nc),
                          eps=1.0 if eps is None else eps, eps_cells=e, alpha=1.0, trunc=T.ADAPTIVE, m_init=2,
                          m_cap=64, particle_weight=w, uid=8000 + nc, seed=seed, precision=T.FP32_MIXED)
        ctx = T.Context([inst], [T.device_particles(vx, vy, vz, x, T.FP32_MIXED)])
        ctx.use_graph(True)
        wall, kernel_ms = time_steps(ctx, steps, warmup, True)
        out[name] = {"cells": nc, "particles": len(x), "ms_per_step": wall * 1e3 / steps, "event_ms": kernel_ms,
                     "particle_steps_per_s": len(x) * steps / wall}
        log(f"tube {name}: {out[name]}")
        ctx.close()
        torch.cuda.empty_cache()
    return out


def serving(T, args):
    """Serving: a Poisson stream of homogeneous solves and shock tubes (N
    log-uniform in [1e3, 1e6], 50-500 steps, eps log-uniform in [1e-4, 1]) served
    with continuous batching under an HBM budget, arrivals in real time; then the
    same requests all queued at time 0 (the saturation run: the served form's
    throughput when the GPU never waits for arrivals)."""
    import torch

    import workloads as W
    from paper_1009_2768_amd.serve import Server, summarize
    reqs = W.serving_requests(args.serve_rate, args.serve_seconds, seed=args.seed)
    log(f"serving {len(reqs)} requests over {args.serve_seconds} s ...")
    names = ["default", "group", "wave", "tiled"]
    out = {"rate_per_s": args.serve_rate, "stream_s": args.serve_seconds, "hbm_budget_gib": args.serve_budget_gib,
           "precision": "fp32", "ticks_ahead": args.serve_ahead,
           "mix": "homogeneous solves (Maxwell / hard spheres 50/50, BKW / bi-Maxwellian 50/50) and Sod tubes "
                  "(hard spheres, 888 / 111 particles per cell) 50/50, N log-uniform [1e3, 1e6], 50-500 steps, "
                  "eps log-uniform [1e-4, 1]"}
    table = None
    for name, realtime in (("poisson", True), ("saturation", False)):
        srv = Server(hbm_budget=int(args.serve_budget_gib * 2**30), max_instances=4096, max_cells=1 << 21)
        if table is None:
            t0 = time.time()
            table, _ = srv.tune(reqs, log=log)  # outside the served stream
            log(f"serving schedule tuned in {time.time() - t0:.1f} s")
            out["schedule"] = {f"2^{b}": names[p] for b, p in enumerate(table) if p}
        else:
            srv.ctx.set_schedule(table)
        done = srv.run(reqs, realtime=realtime, ahead=args.serve_ahead)
        srv.close()
        res = summarize(done, srv.wall, srv.busy)
        res.update({"peak_hbm_gib": srv.peak_bytes / 2**30, "peak_running": srv.peak_active, "ticks": srv.ticks})
        out[name] = res
        log(f"serving {name}: p50 {res['p50_ms']:.1f} ms, p99 {res['p99_ms']:.1f} ms, "
            f"{res['particle_steps_per_s']:.3e} particle-steps/s, wall {srv.wall:.2f} s, device busy "
            f"{srv.busy:.2f} s, HBM fraction {res['hbm_frac_wall']:.4f} (wall) {res['hbm_frac_busy']:.4f} (busy)")
        del srv, done
        torch.cuda.empty_cache()
    # the headline figures of the served form: latency at the stated rate, HBM
    # fraction over the device-busy time and at saturation
    out.update({"p50_ms": out["poisson"]["p50_ms"], "p99_ms": out["poisson"]["p99_ms"],
                "particle_steps_per_s": out["poisson"]["particle_steps_per_s"],
                "hbm_frac_busy": out["poisson"]["hbm_frac_busy"],
                "saturation_particle_steps_per_s": out["saturation"]["particle_steps_per_s"],
                "saturation_hbm_frac": out["saturation"]["hbm_frac_wall"]})
    return out


def precision_c4(T, seed, steps=500, every=10, average_from=250):
    """FP32-mixed against FP64 on the transition-regime tube (10^4 cells, 1778 / 222
    particles per cell, about 10^7 particles, eps(x) log-linear from 1e-4 to 1,
    hard spheres, adaptive depth, dt = CFL 0.5), 500 steps from the same initial
    particles.  FP64 stands for the oracle, which it matches to 1e-12 at this size
    (one step, tests).  The two precisions draw the same keyed random numbers but
    their trajectories part within a few steps (a rounding moves an integer
    decision), so the per-cell differences are compared with two FP64 runs of
    different seeds (the noise floor).  Per cell moment (density, u_x over the
    thermal speed, T, P_xx): median / 99th percentile / largest relative
    difference, at the last step and averaged over the steps from average_from on."""
    import numpy as np
    import torch

    import workloads as W
    nc = 10000
    x, vx, vy, vz, w = W.sod(nc, 1778, 222, seed=seed)
    e = W.transition_eps(nc)

    def run(precision, sd):
        inst = T.Instance(n_particles=len(x), geometry=T.SLAB1D, n_cells=nc, dt=W.sod_dt(1.0, nc), eps=1.0,
                          eps_cells=e, alpha=1.0, trunc=T.ADAPTIVE, m_init=2, m_cap=64, particle_weight=w,
                          uid=9000, seed=sd, precision=precision)
        ctx = T.Context([inst], [T.device_particles(vx, vy, vz, x, precision)])
        ctx.use_graph(True)
        acc, k = None, 0
        t0 = time.perf_counter()
        for s in range(steps // every):
            ctx.step(every)
            if (s + 1) * every > average_from:
                m = ctx.moments(0)
                cur = np.stack([m["rho"], m["ux"] / np.sqrt(np.maximum(m["T"], 1e-300)), m["T"], m["Pxx"]])
                acc = cur if acc is None else acc + cur
                k += 1
        ctx.sync()
        wall = time.perf_counter() - t0
        ctx.close()
        torch.cuda.empty_cache()
        return cur, acc / k, wall

    f32, f32avg, w32 = run(T.FP32_MIXED, seed)
    f64, f64avg, w64 = run(T.FP64, seed)
    g64, g64avg, _ = run(T.FP64, seed + 1)
    names = ["rho", "ux_over_thermal_speed", "T", "Pxx"]

    def stats(a, b):
        out = {}
        for j, nm in enumerate(names):
            d = np.abs(a[j] - b[j]) / (1.0 if j == 1 else np.abs(b[j]))
            out[nm] = {"median": float(np.median(d)), "p99": float(np.quantile(d, 0.99)), "max": float(d.max())}
        return out

    return {"workload": f"transition-regime tube, {nc} cells, {len(x)} particles, eps(x) 1e-4..1, hard spheres, "
                        f"adaptive depth, {steps} steps",
            "fp32_vs_fp64_last_step": stats(f32, f64), "fp64_vs_fp64_other_seed_last_step": stats(g64, f64),
            "fp32_vs_fp64_time_averaged": stats(f32avg, f64avg),
            "fp64_vs_fp64_other_seed_time_averaged": stats(g64avg, f64avg),
            "averaged_over": f"every {every}th step from step {average_from + every} to {steps}",
            "fp32_s": w32, "fp64_s": w64}


LEGS_DEFAULT = ("cpu", "batching", "serving", "precision")
LEGS_ALL = LEGS_DEFAULT + ("fusion", "reuse", "shock", "tubes", "wb")


class Line:
    """The one JSON line: filled leg by leg, printed once (at the end, or by the
    watchdog when the run outlives its time budget, with the legs not reached
    listed under "skipped")."""

    def __init__(self):
        import threading
        self.d = {}
        self.lock = threading.Lock()
        self.printed = False
        self.pending = []

    def emit(self):
        with self.lock:
            if self.printed:
                return
            self.printed = True
            if self.pending:
                self.d["skipped"] = list(self.pending)
            print(json.dumps(self.d), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--instances", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--legs", default=",".join(LEGS_DEFAULT),
                    help="legs after the headline, comma-separated, from: " + ",".join(LEGS_ALL) +
                         " ('all' for every one, 'none' for the headline only)")
    ap.add_argument("--budget", type=float, default=420.0,
                    help="seconds after which the line is printed with the legs not yet run listed as skipped")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--path", choices=["auto", "default", "group", "wave", "tiled"], default="auto",
                    help="kernel path per cell: auto = autotuned per size bucket (outside the timed region)")
    ap.add_argument("--table", default=None,
                    help="fixed schedule instead of tuning, e.g. 8:wave,9:wave,11:group (bucket:path)")
    ap.add_argument("--no-graph", action="store_true", help="launch kernels one by one instead of a HIP graph")
    ap.add_argument("--no-fuse", action="store_true",
                    help="one launch per step instead of one launch taking every cell through all timed steps")
    ap.add_argument("--no-order", action="store_true",
                    help="launch cells in the order of expected size instead of their measured step time")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="length of the Poisson request stream")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="mean arrivals per second")
    ap.add_argument("--speedup-stride", type=int, default=16,
                    help="compare batched and one-at-a-time stepping on every n-th instance")
    ap.add_argument("--serve-budget-gib", type=float, default=96.0, help="HBM budget of the running requests")
    ap.add_argument("--serve-ahead", type=int, default=2, help="ticks the serving host may run ahead of the GPU")
    ap.add_argument("--wb-instances", type=int, default=64, help="instances of the tree-shape truncation leg")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB each (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}), flush=True)
        sys.exit(2)
    legs = [] if args.legs == "none" else list(LEGS_ALL) if args.legs == "all" else \
        [s for s in args.legs.split(",") if s]
    for s in legs:
        if s not in LEGS_ALL:
            ap.error(f"unknown leg {s}")

    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n, "copies": 5}), flush=True)
        return

    t_start = time.time()
    out = Line()

    import paper_1009_2768_amd as T
    T.load()
    prec = T.FP32_MIXED if args.precision == "fp32" else T.FP64
    N, eps, alpha, init = make_batch(args.instances, args.seed)
    total = int(N.sum())
    log(f"building {args.instances} instances, {total} particles")
    t0 = time.time()
    ctx, bufs = build_context(T, N, eps, alpha, init, args.seed, prec)
    log(f"context ready in {time.time() - t0:.1f} s")
    names = ["default", "group", "wave", "tiled"]
    if args.table:
        table = [0] * T.SCHED_BUCKETS
        for item in args.table.split(","):
            b, name = item.split(":")
            table[int(b)] = names.index(name)
    elif args.path == "auto":
        from paper_1009_2768_amd.autotune import autotune
        t0 = time.time()
        table, _ = autotune(ctx.instances, ctx._particles, log=log)
        log(f"autotune done in {time.time() - t0:.1f} s")
    else:
        table = [names.index(args.path)] * T.SCHED_BUCKETS
    ctx.set_schedule(table)
    schedule = {f"2^{T.size_bucket(i)}": names[table[T.size_bucket(i)]] for i in ctx.instances}
    schedule = dict(sorted(schedule.items(), key=lambda kv: int(kv[0][2:])))
    if not args.no_graph:
        ctx.use_graph(True)
    ctx.order_by_cost(not args.no_order)
    fuse = not args.no_fuse
    log(f"timing {args.steps} steps after {args.warmup} ...")
    wall, avg_ms = time_steps(ctx, args.steps, args.warmup, fuse)
    ms_per_step = wall * 1000.0 / args.steps
    value = total * args.steps / wall
    sz = 4 if prec == T.FP32_MIXED else 8
    algo_bytes = 6 * sz * total  # one read and one write of (vx, vy, vz) per particle-step
    achieved = algo_bytes / (avg_ms * 1e-3) / 1e9  # per step; a fused launch is `steps` steps
    kernel = "k_collide<float>" if prec == T.FP32_MIXED else "k_collide<double>"
    # a cell on the tile pipeline: TILED, or the library default from 2^16 particles on
    tiled = any(table[T.size_bucket(i)] == 3 or (table[T.size_bucket(i)] == 0 and T.size_bucket(i) >= 16)
                for i in ctx.instances)
    fuse = fuse and not tiled  # a cell on the tile pipeline keeps one launch sequence per step
    per_launch = args.steps if fuse else 1
    traffic = None if tiled else stored_traffic(kernel, table, per_launch)
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, kernel events {avg_ms:.3f} ms")
    work = work_totals(T, ctx)
    ctx.close()
    del ctx, bufs
    torch.cuda.empty_cache()
    out.d.update({
        "metric": "particle-collision-step updates/sec",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64sums" if prec == T.FP32_MIXED else "f64",
        "data": "synthetic (BKW / bi-Maxwellian initial data, seeded)",
        "config": {"workload": "batched homogeneous TRMC-R: 4096 instances, N log-uniform [256, 65536], "
                               "eps log-uniform [1e-4, 10], Maxwell/hard-sphere 50/50, adaptive depth m_cap 64, "
                               "dt 0.05",
                   "instances": args.instances, "particles": total, "precision": args.precision,
                   "schedule": schedule, "graph": not args.no_graph, "fused_steps": fuse,
                   "launch_order": "size" if args.no_order else "measured step time"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_schedule": json.load(open(TRAFFIC_RECORD))["table"] if traffic else None,
                     "traffic_counted": None if tiled else traffic_record(kernel),
                     "steps_per_launch": per_launch,
                     "kernel": (kernel + " (+ k_advance, about 4 us)") if not tiled else
                     "tile pipeline + " + kernel + " (several kernels per step)"},
        "work_last_step": work,
    })
    log(f"headline: {value:.4e} particle-steps/s, roofline frac {achieved / HBM_PEAK_GBS:.4f}")

    # legs after the headline; the watchdog prints the line if they outlive the budget
    import threading
    out.pending = list(legs)

    def watchdog():
        log(f"time budget of {args.budget:.0f} s spent; printing the line without {out.pending}")
        out.emit()
        os._exit(0)

    left = args.budget - (time.time() - t_start)
    timer = threading.Timer(max(1.0, left), watchdog)
    timer.daemon = True
    timer.start()
    for leg in legs:
        log(f"leg {leg} ...")
        t0 = time.time()
        if leg == "cpu":
            res = cpu_baseline(N, eps, alpha, init, args.seed, args.cpu_budget)
            out.d["cpu_baseline"] = res
        elif leg == "batching":
            res = batching_speedup(T, N, eps, alpha, init, args.seed, prec, table, args.speedup_stride)
            out.d["batching"] = res
        elif leg == "serving":
            res = serving(T, args)
            out.d["serving"] = res
        elif leg == "precision":
            res = precision_c4(T, args.seed)
            out.d["precision_transition_tube"] = res
        elif leg == "fusion":
            if not fuse:
                res = {"skipped": "steps are not fused on this schedule"}
            else:
                res = step_fusion(T, N, eps, alpha, init, args.seed, prec, table, args.steps, args.warmup,
                                  ms_per_step)
            out.d["step_fusion"] = res
        elif leg == "reuse":
            reuse = adaptive_reuse(T, N, eps, alpha, init, args.seed, prec, table, args.steps, args.warmup, fuse)
            res = {"recompute": dict(ms_per_step=ms_per_step, kernel_ms=avg_ms, **work),
                   "reuse": reuse, "speedup": ms_per_step / reuse["ms_per_step"]}
            out.d["adaptive_reuse"] = res
        elif leg == "shock":
            res = stationary_shock(T, args.seed)
            out.d["stationary_shock"] = res
        elif leg == "tubes":
            res = tubes(T, args.seed)
            out.d["tubes"] = res
        elif leg == "wb":
            res = tree_shape_truncation(T, args.wb_instances, args.seed)
            out.d["tree_shape_truncation"] = res
        out.pending.remove(leg)
        log(f"leg {leg} done in {time.time() - t0:.1f} s: {res}")
    timer.cancel()
    out.emit()


if __name__ == "__main__":
    main()
