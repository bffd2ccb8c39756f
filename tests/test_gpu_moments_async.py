"""GPU: moments written by the device behind the step (trmc_moments_async).

The serving loop reads the results of finished requests without waiting for the
stream: the records land in pinned host memory (or device memory) in stream
order.  They must equal trmc_moments field by field and bit for bit, for a
homogeneous cell and a slab, in FP32 and FP64; a slot retired right after the
call still delivers the records of its last step; a buffer too small for the
slot's cells is refused before anything is enqueued.
"""
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


def make(T, prec):
    vx, vy, vz = W.bkw(5000, 0.6, stream=401)
    homog = T.Instance(n_particles=5000, eps=0.1, alpha=1.0, trunc=T.ADAPTIVE, uid=41, precision=prec)
    x, sx, sy, sz, w = W.sod(40, 60, 20, seed=0, stream=402)
    slab = T.Instance(n_particles=len(x), geometry=T.SLAB1D, n_cells=40, eps=0.01, alpha=1.0,
                      dt=W.sod_dt(1.0, 40), particle_weight=w, trunc=T.ADAPTIVE, uid=42, precision=prec)
    parts = [T.device_particles(vx, vy, vz, None, prec), T.device_particles(sx, sy, sz, x, prec)]
    return T.Context([homog, slab], parts), [1, 40]


def same(a, b, tag):
    assert sorted(a) == sorted(b), tag
    for key in b:
        assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), (tag, key)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_async_records_equal_sync_moments(trmc, prec):
    import torch
    T = trmc
    p = T.FP64 if prec == "fp64" else T.FP32_MIXED
    say("async moments", prec)
    ctx, ncs = make(T, p)
    ctx.step(3)
    for slot, nc in enumerate(ncs):
        ref = ctx.moments(slot)
        host = torch.empty(T.moments_record_bytes(nc), dtype=torch.uint8, pin_memory=True)
        ctx.moments_async(slot, host)
        ctx.sync()
        same(T.unpack_moments(host, nc), ref, ("pinned", slot))
        dev = torch.empty(T.moments_record_bytes(nc), dtype=torch.uint8, device="cuda")
        ctx.moments_async(slot, dev)
        ctx.sync()
        same(T.unpack_moments(dev.cpu(), nc), ref, ("device", slot))
        assert int(ref["n"].sum()) == ctx.instance(slot).n_particles
    # retired right after the call: the records of its last step still arrive
    ref = ctx.moments(1)
    host = torch.empty(T.moments_record_bytes(40), dtype=torch.uint8, pin_memory=True)
    ctx.moments_async(1, host)
    ctx.retire(1)
    ctx.step(2)  # the other instance goes on
    ctx.sync()
    same(T.unpack_moments(host, 40), ref, "retired")
    # a buffer shorter than the slot's cells is refused
    small = torch.empty(T.moments_record_bytes(1), dtype=torch.uint8, pin_memory=True)
    ctx.step(1)
    ctx.sync()
    with pytest.raises(T.TrmcError):
        ctx2, _ = make(T, p)
        try:
            ctx2.moments_async(1, small)
        finally:
            ctx2.close()
    ctx.close()
