"""Serving loop: continuous batching of TRMC-R solves on one GPU.

Requests (homogeneous solves and shock tubes of different sizes, eps and step
counts) arrive over time.  All running requests share one context and advance
together, one step per tick (one trmc_step over every active instance).  At each
tick boundary the loop

  * retires the requests whose last step has run: their moments are written by
    the device into pinned host memory behind the step (trmc_moments_async), the
    slot leaves the active set at once, and the request's device memory is
    released when an event recorded after the copy has passed (checked at every
    tick, so the host never waits for the device to drain),
  * admits waiting requests in arrival order while the HBM budget (particle
    arrays plus library workspace of the running requests) and the slot and
    cell capacities allow,

so requests that arrive while others are on the GPU join the running batch as
soon as memory frees up.  Particle state stays on the device from admission to
retirement.  A request's result does not depend on what it ran with: the
library keys every random draw by (seed, uid, cell, step) and every cell's step
reads only that cell.

Latency is measured from a request's arrival to the moment its results are on
the host; throughput is particle-steps completed per second of wall time.
"""
from __future__ import annotations

import ctypes
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import _abi
from . import (ADAPTIVE, FP32_MIXED, FP64, HOMOG, SLAB1D, Context, Instance, TrmcError, check,
               moments_record_bytes, unpack_moments)


def instance_of(req, precision=FP32_MIXED, m_cap=64) -> Instance:
    """Descriptor of a request (see workloads.serving_requests)."""
    if req["slab"]:
        nc = int(req["n_cells"])
        dx = 1.0 / nc
        return Instance(n_particles=int(req["n"]), geometry=SLAB1D, n_cells=nc, length=1.0,
                        dt=0.5 * dx / 3.0, particle_weight=dx / int(req["ppc_left"]), eps=float(req["eps"]),
                        alpha=float(req["alpha"]), trunc=ADAPTIVE, m_cap=m_cap, precision=precision,
                        seed=int(req["seed"]), uid=int(req["rid"]))
    n = int(req["n"])
    return Instance(n_particles=n, eps=float(req["eps"]), alpha=float(req["alpha"]), dt=0.05,
                    particle_weight=1.0 / n, trunc=ADAPTIVE, m_cap=m_cap, precision=precision,
                    seed=int(req["seed"]), uid=int(req["rid"]))


def workspace_bytes(inst: Instance) -> int:
    d = inst.to_c()
    n = ctypes.c_size_t(0)
    check(_abi.load().trmc_workspace_size(ctypes.byref(d), 1, ctypes.byref(n)), "trmc_workspace_size")
    return int(n.value)


@dataclass
class Done:
    rid: int
    n: int
    steps: int
    arrival: float
    admitted: float
    finished: float
    moments: dict = field(repr=False)
    state: dict | None = field(default=None, repr=False)
    tick_admitted: int = 0
    bytes_per_step: int = 0  # algorithmic HBM bytes of one step: read and write of (x,) v

    @property
    def latency(self):
        return self.finished - self.arrival


class Server:
    """One context, a FIFO queue and an HBM budget for the running requests."""

    def __init__(self, hbm_budget: int, max_instances: int = 4096, max_cells: int = 1 << 20,
                 precision=FP32_MIXED, initial=None, capture=()):
        import torch
        self.precision = precision
        self.dtype = torch.float32 if precision == FP32_MIXED else torch.float64
        self.budget = int(hbm_budget)
        self.ctx = Context([], [], max_instances=max_instances, max_cells=max_cells)
        self.max_instances, self.max_cells = max_instances, max_cells
        if initial is None:
            import workloads
            initial = workloads.serving_initial
        self.initial = initial
        self.capture = set(capture)  # rids whose final particles are read back
        self.used = 0
        self.cells = 0
        self.active = {}  # slot -> [req, steps_left, bytes, t_admit, tensors, tick_admit]
        # retired requests whose results are on their way to the host:
        # [req, bytes, t_admit, tensors, tick_admit, host buffer, event]
        self.draining = deque()
        self.pinned = []  # free pinned host buffers for the results
        self.peak_bytes = 0
        self.peak_active = 0
        self.ticks = 0

    def tune(self, requests, per_bucket: int | None = None, max_particles: int = 8_000_000, refine: bool = True,
             mix_particles: int | None = 100_000_000, log=None):
        """Choose the kernel path per cell-size bucket with the autotuner (before
        serving), timed on copies of the requests of each bucket, up to
        max_particles particles (and per_bucket requests, if given) per bucket.
        The sample is sized for throughput: with only a few requests a bucket
        is timed by its latency alone, where the workgroup per cell wins, while
        a served mix runs many of them at once, where a bucket of many small
        cells runs faster one wave per cell.  refine: then refine the table on
        the requests as one mix (autotune.refine_for_mix; up to mix_particles
        particles, in arrival order), where the buckets share the GPU."""
        from . import size_bucket
        from .autotune import autotune
        picked, count, total = [], {}, {}
        for r in requests:
            inst = instance_of(r, self.precision)
            b = size_bucket(inst)
            if per_bucket is not None and count.get(b, 0) >= per_bucket:
                continue
            if count.get(b, 0) and total[b] + inst.n_particles > max_particles:
                continue
            count[b] = count.get(b, 0) + 1
            total[b] = total.get(b, 0) + inst.n_particles
            picked.append((inst, r))
        insts = [i for i, _ in picked]
        parts = [self.initial(r, dtype=self.dtype) for _, r in picked]
        table, timings = autotune(insts, parts, warmup=1, steps=2, max_particles=max_particles, log=log)
        if refine:
            from .autotune import refine_for_mix
            mix = [(instance_of(r, self.precision), r) for r in requests]
            if mix_particles is not None:
                kept, tot = [], 0
                for inst, r in mix:
                    if tot + inst.n_particles <= mix_particles:
                        kept.append((inst, r))
                        tot += inst.n_particles
                mix = kept
            del parts
            table = refine_for_mix([i for i, _ in mix], [self.initial(r, dtype=self.dtype) for _, r in mix], table,
                                   log=log)
        self.ctx.set_schedule(table)
        self.schedule = table
        return table, timings

    def cost(self, req):
        inst = instance_of(req, self.precision)
        sz = 4 if self.precision == FP32_MIXED else 8
        arrays = (4 if req["slab"] else 3) * sz * int(req["n"])
        return inst, arrays + workspace_bytes(inst)

    def fits(self, req, nbytes):
        cells = int(req["n_cells"]) if req["slab"] else 1
        return (self.used + nbytes <= self.budget and len(self.active) < self.max_instances
                and self.cells + cells <= self.max_cells)

    def admit(self, req, inst, nbytes, now):
        """Admit a request (its memory was checked by fits()); None when the
        library's own budget check (trmc_admit, active instances only) refuses it."""
        parts = self.initial(req, dtype=self.dtype)
        try:
            slot = self.ctx.admit(inst, parts)
        except TrmcError as e:
            if e.code == _abi.EBUSY:
                return None
            raise
        self.active[slot] = [req, int(req["steps"]), nbytes, now, parts, self.ticks]
        self.used += nbytes
        self.cells += int(req["n_cells"]) if req["slab"] else 1
        self.peak_bytes = max(self.peak_bytes, self.used)
        self.peak_active = max(self.peak_active, len(self.active))
        return slot

    def _done(self, req, t_adm, tick, t, mom, state):
        self.cells -= int(req["n_cells"]) if req["slab"] else 1
        sz = 4 if self.precision == FP32_MIXED else 8
        per = (8 if req["slab"] else 6) * sz * int(req["n"])
        return Done(req["rid"], int(req["n"]), int(req["steps"]), req["arrival"], t_adm, t, mom, state, tick, per)

    def retire(self, slot, t0):
        """Take a finished request out of the active set.  Its results are copied
        behind its last step; harvest() returns the request once they are on the
        host.  (A request whose final particles are captured is read at once.)"""
        import torch
        req, _, nbytes, t_adm, parts, tick = self.active.pop(slot)
        if req["rid"] in self.capture:
            mom = self.ctx.moments(slot)  # synchronises: the results are on the host
            state = self.ctx.read(slot)
            t = time.perf_counter() - t0
            self.ctx.retire(slot)
            self.used -= nbytes
            return self._done(req, t_adm, tick, t, mom, state)
        nc = int(req["n_cells"]) if req["slab"] else 1
        need = moments_record_bytes(nc)
        buf = None
        for k, b in enumerate(self.pinned):
            if b.numel() >= need:
                buf = self.pinned.pop(k)
                break
        if buf is None:
            buf = torch.empty(max(need, 1 << 16), dtype=torch.uint8, pin_memory=True)
        self.ctx.moments_async(slot, buf)
        ev = torch.cuda.Event()
        ev.record(self.ctx.stream)
        self.ctx.retire(slot)  # the next step leaves it out; its memory lives until ev
        self.draining.append([req, nbytes, t_adm, parts, tick, buf, ev])
        return None

    def harvest(self, t0, wait=False):
        """Requests whose results have reached the host (in retirement order);
        wait: block for all of them."""
        out = []
        while self.draining and (wait or self.draining[0][6].query()):
            req, nbytes, t_adm, parts, tick, buf, ev = self.draining.popleft()
            ev.synchronize()
            nc = int(req["n_cells"]) if req["slab"] else 1
            mom = unpack_moments(buf, nc)
            t = time.perf_counter() - t0
            self.pinned.append(buf)
            self.used -= nbytes
            out.append(self._done(req, t_adm, tick, t, mom, None))
        return out

    def run(self, requests, realtime: bool = True, log=None, ahead: int = 2):
        """Serve the requests (sorted by arrival).  realtime: arrivals follow the
        wall clock (idle gaps are waited out); otherwise every request is queued
        at time 0.  ahead: ticks the host may run ahead of the device (it prepares
        the next tick while the device runs the current one, and admissions join
        at most that many ticks later).  Returns the list of Done records in
        completion order."""
        import torch
        self.ctx.set_budget(self.budget)  # the library refuses admissions beyond it too (TRMC_EBUSY)
        ticks_ev = []  # (start, end) events of every tick on the context's stream
        pending = deque(sorted(requests, key=lambda r: r["arrival"]))
        waiting = deque()
        done = []
        t0 = time.perf_counter()
        head = None  # (inst, bytes) of waiting[0]
        while pending or waiting or self.active or self.draining:
            done.extend(self.harvest(t0))
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0]["arrival"] <= now):
                r = pending.popleft()
                if not realtime:
                    r = dict(r, arrival=0.0)
                waiting.append(r)
            # admission at the tick boundary, in arrival order
            while waiting:
                if head is None:
                    head = self.cost(waiting[0])
                inst, nbytes = head
                if not self.fits(waiting[0], nbytes) or self.admit(waiting[0], inst, nbytes, now) is None:
                    if not self.active and not self.draining:
                        raise RuntimeError(f"request {waiting[0]['rid']} does not fit in an empty server")
                    break
                waiting.popleft()
                head = None
            if not self.active:
                if self.draining:
                    done.extend(self.harvest(t0, wait=True))
                elif pending:
                    time.sleep(max(0.0, pending[0]["arrival"] - (time.perf_counter() - t0)))
                continue
            ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            ev[0].record(self.ctx.stream)
            self.ctx.step(1)
            ev[1].record(self.ctx.stream)
            ticks_ev.append(ev)
            self.ticks += 1
            if len(ticks_ev) > ahead:
                ticks_ev[-1 - ahead][1].synchronize()
            finished = []
            for slot, st in self.active.items():
                st[1] -= 1
                if st[1] == 0:
                    finished.append(slot)
            for slot in finished:
                d = self.retire(slot, t0)
                if d is not None:
                    done.append(d)
            if log and finished:
                log(f"t={time.perf_counter() - t0:.3f}s tick {self.ticks}: {len(finished)} done, "
                    f"{len(self.active)} running, {len(waiting)} waiting, {self.used / 2**30:.2f} GiB")
        self.wall = time.perf_counter() - t0
        self.ctx.sync()
        self.busy = sum(a.elapsed_time(b) for a, b in ticks_ev) * 1e-3  # device time of the ticks, s
        return done

    def close(self):
        self.ctx.close()


def summarize(done, wall, busy=None, peak_bytes_per_s=8e12):
    """Latency percentiles, throughput, and the HBM roofline fraction of the
    served work (algorithmic bytes: one read and one write of each particle per
    step) over the wall time and over the device-busy time of the ticks."""
    lat = np.array([d.latency for d in done]) * 1e3
    ps = sum(d.n * d.steps for d in done)
    nbytes = float(sum(d.bytes_per_step * d.steps for d in done))
    out = {"requests": len(done), "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
           "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
           "mean_ms": float(lat.mean()) if len(lat) else None,
           "particle_steps_per_s": ps / wall if wall > 0 else None, "particle_steps": ps, "wall_s": wall,
           "hbm_frac_wall": nbytes / wall / peak_bytes_per_s if wall > 0 else None}
    if busy:
        out.update({"device_busy_s": busy, "hbm_frac_busy": nbytes / busy / peak_bytes_per_s})
    return out
