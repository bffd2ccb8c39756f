"""Pins of the open slab of the stationary shock (Sec. 5.2, reading R17).

* The reservoir states satisfy the Rankine-Hugoniot relations the paper prints
  (equal fluxes of mass, momentum and energy), with the closed-form jump of a
  Mach-3 monatomic shock (density x3, pressure x11, temperature x11/3).
* The inward normal speed of an entering particle inverts the flux-weighted
  half-range distribution: its distribution function, by numerical quadrature,
  at the returned speed equals the uniform drawn.
* The expected number of entering particles equals the quadrature of the flux,
  and an empty slab fills at that rate.
* Run long enough, the slab holds the shock: far from it, the time-averaged
  density and temperature are the two Rankine-Hugoniot states.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import workloads as W

GAMMA = 5.0 / 3.0


def test_reservoir_states_satisfy_rankine_hugoniot():
    (r1, u1, T1), (r2, u2, T2) = W.shock_states(3.0, GAMMA)
    p1, p2 = r1 * T1, r2 * T2
    E1 = 0.5 * r1 * u1**2 + p1 / (GAMMA - 1)
    E2 = 0.5 * r2 * u2**2 + p2 / (GAMMA - 1)
    assert r1 * u1 == pytest.approx(r2 * u2, rel=1e-14)
    assert r1 * u1**2 + p1 == pytest.approx(r2 * u2**2 + p2, rel=1e-14)
    assert u1 * (E1 + p1) == pytest.approx(u2 * (E2 + p2), rel=1e-14)
    assert u1 / math.sqrt(GAMMA * T1) == pytest.approx(3.0, rel=1e-15)
    assert (r2 / r1, p2 / p1, T2 / T1) == pytest.approx((3.0, 11.0, 11.0 / 3.0), rel=1e-13)


@pytest.mark.parametrize("a", [3.8729833, 1.0, 0.0, -0.6741999, -2.0])
def test_flux_speed_inverts_the_half_range_flux_law(orc, a):
    dens = lambda t: t * stats.norm.pdf(t - a)  # noqa: E731
    Z = integrate.quad(dens, 0, np.inf, epsabs=0, epsrel=1e-13)[0]
    for u in (1e-6, 0.01, 0.2, 0.5, 0.77, 0.95, 0.999999):
        w = orc.flux_inverse(a, u)
        F = integrate.quad(dens, 0, w, epsabs=0, epsrel=1e-13)[0]
        assert F / Z == pytest.approx(u, abs=1e-10)


@pytest.mark.parametrize("rho,u,T", [(1.0, 3.8729833, 1.0), (3.0, -1.2909944, 11.0 / 3.0), (0.5, 0.0, 2.0)])
def test_inflow_mean_is_the_flux(orc, rho, u, T):
    weight, dt = 1e-4, 1e-3
    s = math.sqrt(T)
    flux = integrate.quad(lambda v: v * stats.norm.pdf(v, loc=u, scale=s), 0, np.inf, epsrel=1e-13)[0]
    assert orc.inflow_mean(rho, u, T, weight, dt) == pytest.approx(rho / weight * flux * dt, rel=1e-10)


def test_empty_slab_fills_at_the_flux_rate(orc):
    up, down = W.shock_states()
    nc, dt, w = 20, 1e-4, 1e-4  # particles cannot cross the slab in one step
    lam = orc.inflow_mean(up[0], up[1], up[2], w, dt) + orc.inflow_mean(down[0], -down[1], down[2], w, dt)
    counts = []
    for k in range(300):
        e = np.zeros(0)
        inst = orc.Instance(e, e, e, x=e, geometry=orc.SLAB, n_cells=nc, dt=dt, eps=1.0, weight=w, bc=orc.BC_INFLOW,
                            in_left=up, in_right=down, capacity=4096, step=k, uid=5)
        inst.run(1)
        counts.append(inst.n)
        xs = inst.x[:inst.n]
        assert np.all((xs >= 0) & (xs <= 1.0))
    # floor(lambda + U) per end: mean lambda, standard deviation at most 1/2 per end
    assert abs(np.mean(counts) - lam) < 4 * 0.71 / math.sqrt(len(counts))


def test_stationary_shock_far_field_states(orc):
    nc, ppc = 50, 300
    x, vx, vy, vz, w, up, down, cap = W.shock(nc, ppc, seed=1)
    inst = orc.Instance(vx, vy, vz, x=x, geometry=orc.SLAB, n_cells=nc, length=1.0, dt=W.shock_dt(1.0, nc),
                        eps=0.1, alpha=1.0, trunc=orc.ADAPTIVE, m_init=2, m_cap=64, weight=w, bc=orc.BC_INFLOW,
                        in_left=up, in_right=down, capacity=cap, seed=1, uid=3)
    rho, T = [], []
    for s in range(400):
        inst.run(1)
        if s >= 200:
            m = inst.moments()
            rho.append(m[:, 0])
            T.append(m[:, 4])
    rho, T = np.mean(rho, 0), np.mean(T, 0)
    assert np.all(np.abs(rho[:5] - up[0]) < 0.03 * up[0]) and np.all(np.abs(T[:5] - up[2]) < 0.03 * up[2])
    assert np.all(np.abs(rho[-8:] - down[0]) < 0.04 * down[0]) and np.all(np.abs(T[-8:] - down[2]) < 0.04 * down[2])
    # the jump sits inside the slab: density rises monotonically on average through it
    assert rho[nc // 4] < 1.2 and rho[3 * nc // 4] > 2.7


def test_open_slab_rejected_without_reservoirs(orc):
    vx, vy, vz = W.bimaxwellian(100, seed=1)
    x = np.linspace(0.01, 0.99, 100)
    with pytest.raises(RuntimeError):
        orc.Instance(vx, vy, vz, x=x, geometry=orc.SLAB, n_cells=4, bc=orc.BC_INFLOW, in_left=(0.0, 1.0, 1.0),
                     in_right=(1.0, 0.0, 1.0), capacity=200).run(1)
