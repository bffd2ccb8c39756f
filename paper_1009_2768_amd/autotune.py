"""Schedule autotuner for batched runs.

The collision step has three kernel paths for a cell (one workgroup, one wave,
or the tile pipeline; trmc_set_schedule).  Which is fastest depends on the cell
size, the depth and the mix, so the tuner measures: the instances are grouped by
schedule bucket (floor(log2) of particles per cell), and for every bucket each
path the bucket's cells can take is timed on copies of that bucket's instances
(a fresh copy per candidate, so every candidate steps the same states).  The
result is a table for Context.set_schedule.  The schedule changes how fast a
run is, and otherwise only the rounding order of the FP64 cell sums (the last
bits; see trmc_set_schedule): a fixed table gives the same bits every run.

A mix whose buckets run together (the served form) is refined afterwards on the
whole mix (refine_for_mix): timed bucket by bucket, a bucket of a few large cells
looks as fast on one workgroup per cell as on the tile pipeline, but in the mix
its long single-workgroup chains lengthen the step of every other request, while
the tile pipeline spreads them over many workgroups on a stream of its own.
"""
from __future__ import annotations

import time
from dataclasses import replace

from . import (HOMOG, PATH_DEFAULT, PATH_GROUP, PATH_TILED, PATH_WAVE, SCHED_BUCKETS, Context, size_bucket)

_SHALLOW = 256  # deepest m_cap of the wave and tile paths


def candidates(insts) -> list[int]:
    paths = [PATH_GROUP]
    if all(i.m_cap <= _SHALLOW for i in insts):
        paths.append(PATH_WAVE)
        if all(i.geometry == HOMOG for i in insts):
            paths.append(PATH_TILED)
    return paths


def _time_path(insts, parts, path, warmup, steps):
    import torch
    clones = [{k: (v.clone() if v is not None else None) for k, v in p.items()} for p in parts]
    ctx = Context([replace(i) for i in insts], clones)
    try:
        ctx.set_schedule([path] * SCHED_BUCKETS)
        ctx.step(warmup)
        ctx.sync()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(ctx.stream):
            a.record(ctx.stream)
            ctx.step(steps)
            b.record(ctx.stream)
        ctx.sync()
        b.synchronize()
        return a.elapsed_time(b) / steps
    finally:
        ctx.close()


def autotune(instances, particles, warmup=1, steps=2, max_particles=8_000_000, margin=0.05, log=None):
    """Return (schedule table, per-bucket timings in ms) for these instances.

    particles[i] holds the device tensors of instances[i]; they are copied, never
    stepped.  At most max_particles particles of a bucket are used to time it.  A
    path other than the workgroup path is chosen only when it is faster by more
    than `margin` (relative).
    """
    buckets: dict[int, list[int]] = {}
    for k, inst in enumerate(instances):
        buckets.setdefault(size_bucket(inst), []).append(k)
    table = [PATH_DEFAULT] * SCHED_BUCKETS
    timings = {}
    for b in sorted(buckets):
        idx, tot = [], 0
        for k in buckets[b]:
            if idx and tot + instances[k].n_particles > max_particles:
                break
            idx.append(k)
            tot += instances[k].n_particles
        insts = [instances[k] for k in idx]
        parts = [particles[k] for k in idx]
        res = {}
        t0 = time.perf_counter()
        for path in candidates(insts):
            res[path] = _time_path(insts, parts, path, warmup, steps)
        # the first candidate (workgroup per cell) stays unless another is clearly
        # faster, so that near-ties do not flip the table from run to run
        best = min(res, key=res.get)
        if res[best] > (1.0 - margin) * res[PATH_GROUP]:
            best = PATH_GROUP
        table[b] = best
        timings[b] = res
        if log:
            log(f"bucket 2^{b}: {len(idx)} instances, {tot} particles: "
                + ", ".join(f"{['default', 'group', 'wave', 'tiled'][p]} {t:.3f} ms" for p, t in res.items())
                + f" -> {['default', 'group', 'wave', 'tiled'][best]} ({time.perf_counter() - t0:.1f} s)")
    return table, timings


def refine_for_mix(instances, particles, table, warmup=2, steps=4, margin=0.03, min_share=0.02, log=None):
    """Coordinate descent of a schedule table on the whole mix: one context holds
    copies of every instance; bucket by bucket (largest share of particles first,
    buckets below min_share of the mix's particles left as they are: their paths
    change a step of the whole mix by less than the timing noise) each other
    path the bucket's cells can take replaces the current one when a step of the
    whole mix is faster by more than `margin`.  The two tables of a
    comparison are timed on the same context in the order current, trial, trial,
    current, and each takes the mean of its two timings, so that a drift of the
    step time over the comparison (the adaptive depths settling) favours neither
    (the copies are thrown away, so they may be stepped under either).  Returns
    the refined table."""
    import torch
    buckets: dict[int, list[int]] = {}
    for k, inst in enumerate(instances):
        buckets.setdefault(size_bucket(inst), []).append(k)
    clones = [{k: (v.clone() if v is not None else None) for k, v in p.items()} for p in particles]
    ctx = Context([replace(i) for i in instances], clones)
    table = list(table)

    def time_of(tab):
        ctx.set_schedule(tab)
        ctx.step(1)  # the rebuilt lists and the graph of this table
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(ctx.stream)
        ctx.step(steps)
        b.record(ctx.stream)
        b.synchronize()
        return a.elapsed_time(b) / steps

    try:
        ctx.set_schedule(table)
        ctx.step(warmup)
        share = {b: sum(instances[k].n_particles for k in buckets[b]) for b in buckets}
        total = sum(share.values())
        order = sorted((b for b in buckets if share[b] >= min_share * total), key=lambda b: -share[b])
        for b in order:
            for path in candidates([instances[k] for k in buckets[b]]):
                if path == table[b]:
                    continue
                trial = list(table)
                trial[b] = path
                a1, b1 = time_of(table), time_of(trial)
                b2, a2 = time_of(trial), time_of(table)
                t_cur, t_new = 0.5 * (a1 + a2), 0.5 * (b1 + b2)
                if log:
                    log(f"mix: bucket 2^{b} {['default', 'group', 'wave', 'tiled'][table[b]]} {t_cur:.3f} ms, "
                        f"{['default', 'group', 'wave', 'tiled'][path]} {t_new:.3f} ms")
                if t_new < (1.0 - margin) * t_cur:
                    table = trial
        ctx.sync()
    finally:
        ctx.close()
    return table
