"""Pins of the oracle's two-stage Runge-Kutta step (the integrator is a reading: the paper
names none; strong-stability-preserving RK2, Heun's method in Shu and Osher's convex form):

    U1 = U + dt F(U, t),  r1 = r + dt v;   U' = U/2 + (U1 + dt F(U1, t + dt))/2,
    r' = r/2 + (r1 + dt v1)/2.

A two-particle step against a 50-digit evaluation of both stages, second-order
self-convergence (the symplectic Euler step converges at first order on the same problem),
conservation of the linear invariants, ballistic motion, the piston's reflection and the
periodic wrap of the final state.
"""
import mpmath as mp
import numpy as np
import pytest

import csph_inputs as ci
from test_oracle_closed_form import (GAMMA, H_SMOOTH, KAPPA, SUPPORT, _mp_state, _pair_state,
                                     _two_particle_rates)


def _rk2_cfg(orc, cfg):
    cfg.integrator = 1
    return cfg


def test_rk2_two_particle_step_by_hand(orc):
    """Both stages in 50 digits: the rates of the pair at U, the predicted pair U1 (positions
    advanced with the OLD velocity), the rates at U1 and the convex combination."""
    mp.mp.dps = 50
    cfg, s = _pair_state(orc, True)
    cfg = _rk2_cfg(orc, cfg)
    dt = 0.1
    s1, t1, dtu, cnt = orc.step(cfg, s, t=2.0, dt_in=dt)
    assert dtu == dt and t1 == 2.1 and cnt.tolist() == [1, 1]
    D = mp.mpf(dt)
    H = mp.mpf(SUPPORT)
    a = [_mp_state(s, i) for i in (0, 1)]
    f = [_two_particle_rates(a[0], a[1], H), _two_particle_rates(a[1], a[0], H)]
    u1 = []
    for i in (0, 1):
        u = dict(a[i])
        for c in ("x", "y", "z"):
            u[c] = a[i][c] + D * a[i]["v" + c]
            u["v" + c] = a[i]["v" + c] + D * f[i]["dv" + c]
        u["rho"] = a[i]["rho"] + D * f[i]["drho"]
        u["E"] = a[i]["E"] + D * f[i]["dE"]
        u1.append(u)
    g = [_two_particle_rates(u1[0], u1[1], H), _two_particle_rates(u1[1], u1[0], H)]
    euler_x = []
    for i in (0, 1):
        want = {}
        for c in ("x", "y", "z"):
            want[c] = a[i][c] / 2 + (u1[i][c] + D * u1[i]["v" + c]) / 2
            want["v" + c] = a[i]["v" + c] / 2 + (u1[i]["v" + c] + D * g[i]["dv" + c]) / 2
        want["rho"] = a[i]["rho"] / 2 + (u1[i]["rho"] + D * g[i]["drho"]) / 2
        want["E"] = a[i]["E"] / 2 + (u1[i]["E"] + D * g[i]["dE"]) / 2
        for k, v in want.items():
            assert abs(s1[k][i] - float(v)) <= 1e-15 * (1 + abs(float(v))), (i, k)
        euler_x.append(float(a[i]["x"] + D * (a[i]["vx"] + D * f[i]["dvx"])))
    # the Euler step lands dt^2-order away, far above rounding
    assert all(abs(s1["x"][i] - euler_x[i]) > 1e-9 for i in (0, 1))


def _smooth_box(orc):
    """Periodic 6^3 lattice with a smooth velocity field (one sine mode per axis)."""
    w = ci.periodic_block(6, 6, 6, seed=21, periodic=7, amp=0.05)
    k = 2 * np.pi / 6.0
    w.vx = 0.05 * np.sin(k * w.y)
    w.vy = 0.05 * np.sin(k * w.z)
    w.vz = 0.05 * np.sin(k * w.x)
    w.p = 1.0 + 0.05 * np.cos(k * w.x)
    return w


def _run(orc, w, integrator, dt, T):
    cfg = orc.cfg_for(w, search=1, cfl=0.0, integrator=integrator)
    s = orc.state_from(w, cfg)
    t = 0.0
    for _ in range(int(round(T / dt))):
        s, t, _, _ = orc.step(cfg, s, t, dt_in=dt)
    return np.concatenate([s[k] for k in ("x", "y", "z", "vx", "vy", "vz", "rho", "E")])


def test_rk2_converges_at_second_order(orc):
    """Self-convergence on a smooth periodic flow to T = 0.8: the differences between runs at
    dt, dt/2, dt/4 shrink 4x per halving for RK2, 2x for the symplectic Euler step."""
    w = _smooth_box(orc)
    T = 0.8
    for integrator, lo, hi in ((1, 3.6, 4.4), (0, 1.8, 2.2)):
        u = [_run(orc, w, integrator, 0.2 / 2 ** k, T) for k in range(4)]
        e = [np.abs(u[k] - u[k + 1]).max() for k in range(3)]
        ratios = [e[k] / e[k + 1] for k in range(2)]
        assert all(lo < r < hi for r in ratios), (integrator, e, ratios)


def test_rk2_conserves_linear_invariants(orc):
    """Closed periodic box: sum m v and sum m E are conserved to round-off (the step is a
    convex combination of forward-Euler stages, each conserving them)."""
    w = ci.periodic_block(8, 8, 8, seed=22, periodic=7, amp=0.3)
    rng = np.random.default_rng(22)
    w.vx, w.vy, w.vz = (rng.uniform(-0.5, 0.5, w.n) for _ in range(3))
    w.p = rng.uniform(0.5, 2.0, w.n)
    cfg = orc.cfg_for(w, search=1, integrator=1)
    s = orc.state_from(w, cfg)
    s1, _, dt, _ = orc.step(cfg, s, 0.0)
    assert dt > 0
    tot0, tot1 = orc.totals(s), orc.totals(s1)
    assert tot1[0] == tot0[0]
    scale = np.abs(s["m"]).sum() * (1 + np.abs(s["E"]).max())
    for k in (1, 2, 3, 4):
        assert abs(tot1[k] - tot0[k]) < 1e-14 * scale, k


@pytest.mark.parametrize("vw", [0.0, 0.5])
def test_rk2_lone_particle_ballistic_reflected_and_wrapped(orc, vw):
    """No partners: the step is r + dt v (to rounding); crossing the piston plane reflects the
    final state as in the Euler step; leaving a periodic face wraps it."""
    one = lambda v: np.array([v], np.float64)
    base = dict(y=one(0.5), z=one(-0.25), vy=one(0.3), vz=one(-0.1), rho=one(1.0), m=one(1.0),
                mat=np.zeros(1, np.int32))
    cfg = orc.make_cfg([(0, GAMMA, 0.0)], h=H_SMOOTH, kappa=KAPPA, cfl=0.0, integrator=1)
    s = dict(base, x=one(8.0), vx=one(-20.0))
    s["E"] = orc.init_energy(cfg, s["rho"], one(1.0), s["vx"], s["vy"], s["vz"], s["mat"])
    s1, _, _, cnt = orc.step(cfg, s, t=1.0, dt_in=0.1)
    assert cnt.tolist() == [0]
    assert abs(s1["x"][0] - 6.0) <= 1e-15 and s1["vx"][0] == -20.0 and s1["E"][0] == s["E"][0]
    cfg = orc.make_cfg([(0, GAMMA, 0.0)], h=H_SMOOTH, kappa=KAPPA, cfl=0.0, integrator=1,
                       wall=(0.0, vw))
    # fast enough that the predicted position (x = -6) lies farther than the support from its
    # own mirror image, so neither stage has a partner
    s = dict(base, x=one(4.0), vx=one(-100.0))
    s["E"] = orc.init_energy(cfg, s["rho"], one(1.0), s["vx"], s["vy"], s["vz"], s["mat"])
    s1, _, _, _ = orc.step(cfg, s, t=1.0, dt_in=0.1)
    xw = vw * 1.1
    assert s1["x"][0] == pytest.approx(2 * xw - (4.0 - 10.0), abs=1e-14)
    assert s1["vx"][0] == 2 * vw + 100.0
    cfg = orc.make_cfg([(0, GAMMA, 0.0)], h=H_SMOOTH, kappa=KAPPA, cfl=0.0, integrator=1,
                       periodic=1, box=((0.0, -10.0, -10.0), (10.0, 10.0, 10.0)))
    s = dict(base, x=one(0.3), vx=one(-5.0))
    s["E"] = orc.init_energy(cfg, s["rho"], one(1.0), s["vx"], s["vy"], s["vz"], s["mat"])
    s1, _, _, _ = orc.step(cfg, s, t=0.0, dt_in=0.1)
    assert s1["x"][0] == pytest.approx(0.3 - 0.5 + 10.0, abs=1e-14)
