"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module draws initial particle states and instance parameters only; it holds
none of the collision method's arithmetic.  All generators use numpy's PCG64 with
an explicit seed so that both sides of a parity test start from identical arrays.

Initial data (the paper's own tests use sums of Maxwellians and a Rankine-Hugoniot
shock; its data files are not available, so these synthetic recipes stand in):
  - BKW: the Bobylev / Krook-Wu similarity solution for Maxwell molecules at
    shape parameter K (mass 1, zero mean, temperature 1);
  - bi-Maxwellian: two unit-temperature Gaussians with means +-(1, 0, 0);
  - Sod-type slab: left half density 1 / temperature 1, right half density 0.125 /
    temperature 0.8, positions uniform inside each cell.
"""
from __future__ import annotations

import math

import numpy as np


def rng(seed: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed), int(stream)]))


def bkw(n: int, K: float = 0.6, seed: int = 0, stream: int = 0):
    """Velocities from the BKW density with shape K (3/5 <= K <= 1).

    f = G_K(v) [ (5K-3)/(2K) + (1-K)|v|^2/(2K^2) ] with G_K the N(0, K I) density:
    with probability (5K-3)/(2K) a N(0, K I) sample, otherwise an isotropic sample
    with |v|^2 / K distributed chi-square with 5 degrees of freedom.
    """
    g = rng(seed, stream)
    p_gauss = (5.0 * K - 3.0) / (2.0 * K)
    gauss = g.random(n) < p_gauss
    v = g.standard_normal((n, 3)) * math.sqrt(K)
    m = int((~gauss).sum())
    if m:
        r = np.sqrt(K * g.chisquare(5, m))
        d = g.standard_normal((m, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        v[~gauss] = d * r[:, None]
    return v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy()


def bkw_m4(t_over_eps: float, K0: float = 0.6) -> float:
    """Fourth moment of the BKW solution: 15 K (2 - K), 1 - K(t) = (1 - K0) e^{-t/6}
    for the normalised Maxwell kernel (total collision rate 1 at density 1)."""
    one_minus_K = (1.0 - K0) * math.exp(-t_over_eps / 6.0)
    return 15.0 - 15.0 * one_minus_K * one_minus_K


def bimaxwellian(n: int, seed: int = 0, stream: int = 0):
    """Two unit-temperature Gaussians with means +(1,0,0) (even ids) and -(1,0,0) (odd ids)."""
    g = rng(seed, stream)
    v = g.standard_normal((n, 3))
    sign = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    v[:, 0] += sign
    return v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy()


def shell(n: int, radius: float = 1.0, seed: int = 0, stream: int = 0):
    """Velocities uniform on a sphere of the given radius, shifted to zero mean: every
    particle starts near the largest distance from the mean, so collisions push some
    beyond it (a case that exceeds the step's VHS majorant sigma(2 dv))."""
    g = rng(seed, stream)
    d = g.standard_normal((n, 3))
    d *= radius / np.linalg.norm(d, axis=1, keepdims=True)
    d -= d.mean(0)
    return d[:, 0].copy(), d[:, 1].copy(), d[:, 2].copy()


def maxwellian(n: int, u=(0.0, 0.0, 0.0), T: float = 1.0, seed: int = 0, stream: int = 0):
    g = rng(seed, stream)
    v = g.standard_normal((n, 3)) * math.sqrt(T) + np.asarray(u)[None, :]
    return v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy()


def sod(n_cells: int, ppc_left: int, ppc_right: int, length: float = 1.0, T_left: float = 1.0,
        T_right: float = 0.8, seed: int = 0, stream: int = 0):
    """Sod-type slab: particles per cell ppc_left on the left half, ppc_right on the right.

    Returns x, vx, vy, vz and the particle weight w = (L / n_cells) / ppc_left, so that
    the left density is 1 and the right density is ppc_right / ppc_left.
    Particles are generated cell by cell, positions uniform in the cell.
    """
    g = rng(seed, stream)
    dx = length / n_cells
    xs, vs = [], []
    for c in range(n_cells):
        left = c < n_cells // 2
        m = ppc_left if left else ppc_right
        T = T_left if left else T_right
        xs.append(c * dx + g.random(m) * dx)
        vs.append(g.standard_normal((m, 3)) * math.sqrt(T))
    x = np.concatenate(xs)
    v = np.concatenate(vs)
    w = dx / ppc_left
    return x, v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy(), w


def sod_dt(length: float, n_cells: int, cfl: float = 0.5, v_ref: float = 3.0) -> float:
    """dt = CFL * dx / v_ref with v_ref = max over the two states of |u| + 3 sqrt(T) = 3."""
    return cfl * (length / n_cells) / v_ref


def shock_states(mach: float = 3.0, gamma: float = 5.0 / 3.0, rho1: float = 1.0, T1: float = 1.0):
    """Upstream and downstream states (rho, u, T) of a stationary normal shock,
    upstream entering along +x: the Rankine-Hugoniot jump of a monatomic gas
    (p = rho T, sound speed sqrt(gamma T))."""
    u1 = mach * math.sqrt(gamma * T1)
    m2 = mach * mach
    r = (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)   # rho2 / rho1
    pr = (2.0 * gamma * m2 - (gamma - 1.0)) / (gamma + 1.0)  # p2 / p1
    rho2 = rho1 * r
    T2 = T1 * pr / r
    return (rho1, u1, T1), (rho2, u1 / r, T2)


def shock(n_cells: int, ppc_up: int, mach: float = 3.0, length: float = 1.0, seed: int = 0, stream: int = 0,
          capacity_factor: float = 1.5):
    """Slab holding a stationary shock at its centre: the upstream state on the left
    half (ppc_up particles per cell), the downstream state on the right half (as many
    particles per cell as its density ratio asks).  Returns x, vx, vy, vz, the
    particle weight, the two states and a capacity for the arrays (room for the
    reservoirs' particles)."""
    up, down = shock_states(mach)
    g = rng(seed, stream)
    dx = length / n_cells
    w = up[0] * dx / ppc_up
    xs, vs = [], []
    for c in range(n_cells):
        rho, u, T = up if c < n_cells // 2 else down
        m = int(round(rho * dx / w))
        xs.append(c * dx + g.random(m) * dx)
        v = g.standard_normal((m, 3)) * math.sqrt(T)
        v[:, 0] += u
        vs.append(v)
    x = np.concatenate(xs)
    v = np.concatenate(vs)
    cap = int(capacity_factor * len(x)) + 4096
    return x, v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy(), w, up, down, cap


def shock_dt(length: float, n_cells: int, cfl: float = 0.5, mach: float = 3.0) -> float:
    """dt = CFL * dx / (u1 + 3 sqrt(T1)) with the upstream state of shock_states."""
    (rho1, u1, T1), _ = shock_states(mach)
    return cfl * (length / n_cells) / (u1 + 3.0 * math.sqrt(T1))


def transition_eps(n_cells: int, lo: float = 1e-4, hi: float = 1.0):
    """eps(x) log-linear from lo to hi across the cells (cell centres)."""
    c = (np.arange(n_cells) + 0.5) / n_cells
    return lo * (hi / lo) ** c


def batched_homogeneous(n_inst: int, seed: int = 0, n_min: int = 256, n_max: int = 65536,
                        eps_min: float = 1e-4, eps_max: float = 10.0):
    """Parameters of a batch of independent homogeneous instances.

    N log-uniform in [n_min, n_max], eps log-uniform in [eps_min, eps_max], Maxwell
    molecules (alpha 0) and hard spheres (alpha 1) alternating, BKW initial data for
    instances with floor(i/2) even and bi-Maxwellian for the others.
    """
    g = rng(seed, 7)
    u1 = g.random(n_inst)
    u2 = g.random(n_inst)
    N = np.rint(n_min * (n_max / n_min) ** u1).astype(np.int64)
    eps = eps_min * (eps_max / eps_min) ** u2
    alpha = (np.arange(n_inst) % 2).astype(np.float64)
    init = np.where((np.arange(n_inst) // 2) % 2 == 0, 0, 1)  # 0 BKW, 1 bi-Maxwellian
    return N, eps, alpha, init


def batched_velocities(N, init, seed: int = 0, K0: float = 0.6):
    """Concatenated initial velocities for the batch (instance i uses stream 1000 + i)."""
    vx, vy, vz = [], [], []
    for i, (n, kind) in enumerate(zip(N, init)):
        a = bkw(int(n), K0, seed, 1000 + i) if kind == 0 else bimaxwellian(int(n), seed, 1000 + i)
        vx.append(a[0]); vy.append(a[1]); vz.append(a[2])
    return np.concatenate(vx), np.concatenate(vy), np.concatenate(vz)


def serving_requests(rate: float, duration: float, seed: int = 0, n_min: int = 1000, n_max: int = 1_000_000,
                     steps_min: int = 50, steps_max: int = 500, eps_min: float = 1e-4, eps_max: float = 1.0,
                     slab_fraction: float = 0.5, ppc_left: int = 888, ppc_right: int | None = None):
    """A Poisson request stream for the serving loop.

    Arrivals with exponential gaps of mean 1/rate over [0, duration); each request
    is a homogeneous solve (Maxwell molecules or hard spheres, 50/50; BKW or
    bi-Maxwellian initial data, 50/50) or a Sod-type shock tube (hard spheres),
    with N log-uniform in [n_min, n_max], a step count uniform in [steps_min,
    steps_max] and eps log-uniform in [eps_min, eps_max].  A tube has ppc_left
    particles per cell on its left half and ppc_right (default ppc_left / 8, the
    density ratio 0.125) on its right half, and an even number of cells
    n_cells = max(2, 2 round(N / (ppc_left + ppc_right))), so that its particle
    count is close to N (888 / 111 particles per cell: n_cells = N / 499.5).
    """
    g = rng(seed, 11)
    ppc_r = max(1, ppc_left // 8) if ppc_right is None else int(ppc_right)
    out, t, rid = [], 0.0, 0
    while True:
        t += g.exponential(1.0 / rate)
        if t >= duration:
            break
        n = int(round(n_min * (n_max / n_min) ** g.random()))
        steps = int(g.integers(steps_min, steps_max + 1))
        eps = float(eps_min * (eps_max / eps_min) ** g.random())
        slab = bool(g.random() < slab_fraction)
        hard = bool(g.random() < 0.5)
        req = {"rid": rid, "arrival": t, "slab": slab, "steps": steps, "eps": eps, "seed": seed,
               "alpha": 1.0 if (slab or hard) else 0.0, "init": int(g.integers(0, 2))}
        if slab:
            nc = int(min(12288, max(2, 2 * round(n / (ppc_left + ppc_r)))))
            left = nc // 2
            req.update(n_cells=nc, ppc_left=ppc_left, ppc_right=ppc_r,
                       n=left * ppc_left + (nc - left) * ppc_r)
        else:
            req.update(n_cells=1, n=n)
        out.append(req)
        rid += 1
    return out


def serving_initial(req, device="cuda", dtype=None):
    """Initial particles of a serving request, drawn on the device with a torch
    generator seeded by (seed, rid): deterministic for a given device, whether the
    request runs alone or in a mix.  Tubes: the Sod states, positions uniform in
    each cell; homogeneous solves: BKW (init 0) or bi-Maxwellian (init 1).
    Returns dict(x, vx, vy, vz) of tensors."""
    import torch
    dtype = dtype or torch.float32
    gen = torch.Generator(device=device)
    gen.manual_seed(int(req["seed"]) * 1_000_003 + int(req["rid"]) + 1)
    n = int(req["n"])
    if req["slab"]:
        nc, left = int(req["n_cells"]), int(req["n_cells"]) // 2
        pl, pr = int(req["ppc_left"]), int(req["ppc_right"])
        counts = torch.tensor([pl] * left + [pr] * (nc - left), device=device)
        cell = torch.repeat_interleave(torch.arange(nc, device=device), counts)
        dx = 1.0 / nc
        x = (cell.to(torch.float64) + torch.rand(n, generator=gen, device=device, dtype=torch.float64)) * dx
        sd = torch.where(cell < left, torch.tensor(1.0, device=device), torch.tensor(math.sqrt(0.8), device=device))
        v = torch.randn(3, n, generator=gen, device=device, dtype=torch.float64) * sd.to(torch.float64)
        return {"x": x.to(dtype), "vx": v[0].to(dtype).contiguous(), "vy": v[1].to(dtype).contiguous(),
                "vz": v[2].to(dtype).contiguous()}
    v = torch.randn(3, n, generator=gen, device=device, dtype=torch.float64)
    if req["init"] == 1:  # bi-Maxwellian: means +-1 along x
        sign = torch.where(torch.arange(n, device=device) % 2 == 0, 1.0, -1.0).to(torch.float64)
        v[0] += sign
    else:
        # BKW at K = 3/5 (the recipe of bkw()): N(0, K I) with probability
        # (5K - 3)/(2K), else radius sqrt(K chi2_5) in a uniform direction
        K = 0.6
        gauss = torch.rand(n, generator=gen, device=device, dtype=torch.float64) < (5.0 * K - 3.0) / (2.0 * K)
        chi2 = torch.randn(5, n, generator=gen, device=device, dtype=torch.float64).square().sum(0)
        d = v / v.norm(dim=0, keepdim=True).clamp_min(1e-300)
        v = torch.where(gauss[None, :], v * math.sqrt(K), d * (K * chi2).sqrt()[None, :])
    return {"x": None, "vx": v[0].to(dtype).contiguous(), "vy": v[1].to(dtype).contiguous(),
            "vz": v[2].to(dtype).contiguous()}
