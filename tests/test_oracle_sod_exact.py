"""The oracle against the exact solution of the Riemann problem (Sod's shock tube).

The exact solution of the one-dimensional Riemann problem for an ideal gas is written out here
from its standard construction: the star pressure p* solves f_L(p) + f_R(p) + u_R - u_L = 0,
where f_K is the shock (Rankine-Hugoniot) branch for p > p_K and the isentropic rarefaction
branch otherwise; u* follows, and the solution at x/t is sampled from the wave pattern (shock,
or rarefaction head, fan and tail, on each side of the contact).  It is pinned to the published
star state of Sod's problem (p* = 0.30313, u* = 0.92745) and to the jump conditions.

The oracle then runs Sod's tube in the workloads' mode (fixed h = 1.5, support 3, jittered
unit lattice, ideal gas 1.4; periodic across the tube so that it is one-dimensional in the
mean) to t ~ 12 with the CFL rule.  What the scheme must reproduce at this resolution: the
shock where the exact solution puts it (within 1.5 spacings: conservation fixes its speed),
the undisturbed states, and the post-shock plateau's pressure and velocity within the
accuracy this smoothing scale allows (measured on the plateau's mean: pressure 10 % low,
velocity 7 % high, the shock 0.3 spacings behind; the acoustic contact flux and the expanded
gas behind the contact, sampled by few layers, smear the star states), plus the exact
conservation of mass and energy.
"""
import numpy as np
import pytest
from scipy.optimize import brentq

import csph_inputs as ci
import oracle as O

GAMMA = 1.4


def _f(p, rho, pk, c):
    """Velocity change across the wave that takes state K to pressure p."""
    if p > pk:
        a, b = 2.0 / ((GAMMA + 1.0) * rho), (GAMMA - 1.0) / (GAMMA + 1.0) * pk
        return (p - pk) * np.sqrt(a / (p + b))
    return 2.0 * c / (GAMMA - 1.0) * ((p / pk) ** ((GAMMA - 1.0) / (2.0 * GAMMA)) - 1.0)


def star(L, R):
    (rl, ul, pl), (rr, ur, pr) = L, R
    cl, cr = np.sqrt(GAMMA * pl / rl), np.sqrt(GAMMA * pr / rr)
    ps = brentq(lambda p: _f(p, rl, pl, cl) + _f(p, rr, pr, cr) + ur - ul, 1e-12, 100.0,
                xtol=1e-15, rtol=1e-15)
    us = 0.5 * (ul + ur) + 0.5 * (_f(ps, rr, pr, cr) - _f(ps, rl, pl, cl))
    return ps, us


def sample(xi, L, R):
    """(rho, u, p) of the exact solution at x/t = xi."""
    (rl, ul, pl), (rr, ur, pr) = L, R
    cl, cr = np.sqrt(GAMMA * pl / rl), np.sqrt(GAMMA * pr / rr)
    ps, us = star(L, R)
    gm = (GAMMA - 1.0) / (GAMMA + 1.0)
    ex = (GAMMA - 1.0) / (2.0 * GAMMA)
    if xi <= us:  # left of the contact
        if ps > pl:
            s = ul - cl * np.sqrt((GAMMA + 1.0) / (2.0 * GAMMA) * ps / pl + ex)
            return (rl, ul, pl) if xi <= s else (rl * (ps / pl + gm) / (gm * ps / pl + 1.0), us, ps)
        if xi <= ul - cl:
            return (rl, ul, pl)
        if xi >= us - cl * (ps / pl) ** ex:
            return (rl * (ps / pl) ** (1.0 / GAMMA), us, ps)
        q = 2.0 / (GAMMA + 1.0) + gm / cl * (ul - xi)
        return (rl * q ** (2.0 / (GAMMA - 1.0)), 2.0 / (GAMMA + 1.0) * (cl + 0.5 * (GAMMA - 1.0) * ul + xi),
                pl * q ** (2.0 * GAMMA / (GAMMA - 1.0)))
    if ps > pr:
        s = ur + cr * np.sqrt((GAMMA + 1.0) / (2.0 * GAMMA) * ps / pr + ex)
        return (rr, ur, pr) if xi >= s else (rr * (ps / pr + gm) / (gm * ps / pr + 1.0), us, ps)
    if xi >= ur + cr:
        return (rr, ur, pr)
    if xi <= us + cr * (ps / pr) ** ex:
        return (rr * (ps / pr) ** (1.0 / GAMMA), us, ps)
    q = 2.0 / (GAMMA + 1.0) - gm / cr * (ur - xi)
    return (rr * q ** (2.0 / (GAMMA - 1.0)), 2.0 / (GAMMA + 1.0) * (-cr + 0.5 * (GAMMA - 1.0) * ur + xi),
            pr * q ** (2.0 * GAMMA / (GAMMA - 1.0)))


SOD_L, SOD_R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)


def test_exact_solution_pins():
    ps, us = star(SOD_L, SOD_R)
    assert abs(ps - 0.30313) < 1e-5 and abs(us - 0.92745) < 1e-5
    # the right shock: mass and momentum fluxes across it agree (Rankine-Hugoniot)
    r2 = sample(us + 1e-9, SOD_L, SOD_R)[0]
    rr, ur, pr = SOD_R
    s = (r2 * us - rr * ur) / (r2 - rr)
    assert abs(r2 * (us - s) - rr * (ur - s)) < 1e-12
    assert abs((r2 * us * (us - s) + ps) - (rr * ur * (ur - s) + pr)) < 1e-12
    # a symmetric collision stops at the contact; identical states give no waves
    assert abs(star((1.0, 1.0, 1.0), (1.0, -1.0, 1.0))[1]) < 1e-12
    assert abs(star(SOD_L, SOD_L)[0] - 1.0) < 1e-12
    # the left fan joins the undisturbed state and the left star state continuously
    cl = np.sqrt(GAMMA)
    assert abs(sample(-cl + 1e-9, SOD_L, SOD_R)[0] - 1.0) < 1e-6
    tail = us - cl * (ps / 1.0) ** ((GAMMA - 1.0) / (2.0 * GAMMA))
    assert abs(sample(tail - 1e-9, SOD_L, SOD_R)[0] - sample(tail + 1e-9, SOD_L, SOD_R)[0]) < 1e-6


@pytest.fixture(scope="module")
def sod_tube():
    w = ci.periodic_block(160, 7, 7, seed=5, periodic=6)
    left = w.x < 80.0
    w.rho = np.where(left, 1.0, 0.125)
    w.p = np.where(left, 1.0, 0.1)
    w.m = w.rho.copy()
    cfg = O.cfg_for(w, search=1)
    s = O.state_from(w, cfg)
    tot0 = O.totals(s)
    t = 0.0
    while t < 12.0:
        s, t, _, _ = O.step(cfg, s, t)
    return s, t, tot0


def test_oracle_sod_tube_against_the_exact_solution(sod_tube):
    s, t, tot0 = sod_tube
    x, rho, u = s["x"], s["rho"], s["vx"]
    p = (GAMMA - 1.0) * rho * (s["E"] - 0.5 * (s["vx"] ** 2 + s["vy"] ** 2 + s["vz"] ** 2))
    ps, us = star(SOD_L, SOD_R)
    r2 = sample(us + 1e-9, SOD_L, SOD_R)[0]  # behind the shock
    x_shock = 80.0 + t * r2 * us / (r2 - 0.125)  # its speed from the mass flux
    # the shock: the last particle (in x) above the mid density of the jump
    mid = 0.5 * (0.125 + r2)
    xs = x[rho > mid].max()
    print(f"shock at {xs:.2f} (exact {x_shock:.2f})")
    assert abs(xs - x_shock) < 1.5, (xs, x_shock)
    # undisturbed gas ahead of the shock and behind the fan head, away from the rarefactions
    # the tube's free ends send in (at the sound speeds of the two gases)
    cr = np.sqrt(GAMMA * 0.1 / 0.125)
    ahead = (x > x_shock + 3.0) & (x < 160.0 - cr * t - 4.0)
    behind = (x > np.sqrt(GAMMA) * t + 4.0) & (x < 80.0 - np.sqrt(GAMMA) * t - 4.0)
    for sel, (r0, u0, p0) in ((ahead, SOD_R), (behind, SOD_L)):
        assert sel.sum() > 500
        assert abs(rho[sel].mean() - r0) < 0.01 * r0
        assert abs(p[sel].mean() - p0) < 0.01 * p0
        assert abs(u[sel].mean() - u0) < 0.01
    # the post-shock plateau between the contact and the shock
    plat = (x > 80.0 + us * t + 3.0) & (x < x_shock - 1.5)
    assert plat.sum() > 200
    print(f"post-shock p {p[plat].mean():.4f} (exact {ps:.4f}), u {u[plat].mean():.4f} "
          f"(exact {us:.4f})")
    assert abs(p[plat].mean() - ps) < 0.2 * ps, p[plat].mean()
    assert abs(u[plat].mean() - us) < 0.15 * us, u[plat].mean()
    # mass and total energy are conserved (compensated sums)
    tot1 = O.totals(s)
    assert abs(tot1[0] - tot0[0]) <= 1e-12 * tot0[0]
    assert abs(tot1[4] - tot0[4]) <= 1e-10 * abs(tot0[4])
