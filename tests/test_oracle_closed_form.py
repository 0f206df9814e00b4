"""More pins of the CPU oracle: two particles in 50-digit arithmetic, a hand-computed
step, the rigid wall that stops particles, the density-change limit of the time step,
the sampled rate evaluation and the cell-list search at cells smaller than the support.

The two-particle references are written from the paper's statement of the method
(sec. 4.1, eqs. SPH:Conti, SPH:Pulse, SPH:Energy) in mpmath at 50 significant
digits, without the oracle's own expressions: the kernel gradient is the numerical
gradient of W(|r_i - r_j|) with respect to r_i, the contact state solves the two
characteristic relations of the acoustic Riemann problem as a linear system, and the
closing speed of the signal speed is minus the rate of change of the pair distance
along the particles' straight paths.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import csph_inputs as ci

GAMMA = 1.4
H_SMOOTH, KAPPA = 1.5, 2.0
SUPPORT = H_SMOOTH * KAPPA


def _wendland(r, H):
    """3D Wendland C2 kernel with support H (the kernel of sec. 4.1, reading R2)."""
    q = r / H
    if q >= 1:
        return mp.mpf(0)
    return 21 / (2 * mp.pi * H ** 3) * (1 - q) ** 4 * (1 + 4 * q)


def _mp_state(s, k):
    return {f: mp.mpf(float(s[f][k])) for f in ("x", "y", "z", "vx", "vy", "vz", "rho", "E", "m")}


def _pressure_sound(p):
    e = p["E"] - (p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2) / 2
    P = (GAMMA - 1) * p["rho"] * e
    return P, mp.sqrt(GAMMA * P / p["rho"])


def _two_particle_rates(a, b, H):
    """Rates and signal speed of particle a interacting with particle b (50 digits)."""
    ra = mp.matrix([a["x"], a["y"], a["z"]])
    rb = mp.matrix([b["x"], b["y"], b["z"]])
    va = mp.matrix([a["vx"], a["vy"], a["vz"]])
    vb = mp.matrix([b["vx"], b["vy"], b["vz"]])
    d = rb - ra
    r = mp.norm(d)
    e = d / r  # e^R from i to j

    # grad_i W_ij: derivative of W(|r_i - r_j|) with respect to each component of r_i
    def w_at(k, h):
        rr = ra.copy()
        rr[k] += h
        return _wendland(mp.norm(rb - rr), H)

    grad = mp.matrix([mp.diff(lambda h, k=k: w_at(k, h), 0) for k in range(3)])
    Pa, ca = _pressure_sound(a)
    Pb, cb = _pressure_sound(b)
    Za, Zb = a["rho"] * ca, b["rho"] * cb
    vL = (va.T * e)[0]
    vR = (vb.T * e)[0]
    # acoustic Riemann problem: P* + Z_L v* = P_L + Z_L v_L, P* - Z_R v* = P_R - Z_R v_R
    sol = mp.lu_solve(mp.matrix([[1, Za], [1, -Zb]]), mp.matrix([Pa + Za * vL, Pb - Zb * vR]))
    ps, vs = sol[0], sol[1]
    Vb = b["m"] / b["rho"]
    e_grad = (e.T * grad)[0]
    drho = 2 * a["rho"] * Vb * (vL - vs) * e_grad
    dv = -(2 / a["rho"]) * Vb * ps * grad
    dE = -(2 / a["rho"]) * Vb * ps * vs * e_grad

    # closing speed: minus the rate of change of |r_j - r_i| along straight paths
    def dist(t):
        return mp.norm((rb + t * vb) - (ra + t * va))

    closing = -mp.diff(dist, 0)
    sig = max(ca, max(ca, cb) + max(mp.mpf(0), closing))
    return dict(drho=drho, dvx=dv[0], dvy=dv[1], dvz=dv[2], dE=dE, signal=sig,
                closing=closing)


def _pair_state(orc, approach):
    """Two ideal-gas particles 1.9 apart along a skew direction, unequal states; the
    velocities make them approach each other (approach = True) or separate."""
    cfg = orc.make_cfg([(0, GAMMA, 0.0)], h=H_SMOOTH, kappa=KAPPA, cfl=0.0)
    dirn = np.array([0.6, -0.48, 0.64])
    dirn /= np.linalg.norm(dirn)
    sgn = 1.0 if approach else -1.0
    s = dict(x=np.array([0.3, 0.3 + 1.9 * dirn[0]]), y=np.array([-0.2, -0.2 + 1.9 * dirn[1]]),
             z=np.array([0.1, 0.1 + 1.9 * dirn[2]]),
             vx=np.array([0.35 * sgn, -0.1 * sgn]), vy=np.array([-0.2 * sgn, 0.15 * sgn]),
             vz=np.array([0.25 * sgn, -0.3 * sgn]), rho=np.array([1.1, 0.7]),
             m=np.array([1.3, 0.8]), mat=np.zeros(2, np.int32))
    s["E"] = orc.init_energy(cfg, s["rho"], np.array([1.2, 0.45]), s["vx"], s["vy"], s["vz"],
                             s["mat"])
    return cfg, s


@pytest.mark.parametrize("approach", [True, False])
def test_two_particle_rates_closed_form(orc, approach):
    """All five rates and the signal speed of both particles of an isolated pair agree with
    the 50-digit evaluation of the paper's equations; for an approaching pair the signal
    speed exceeds the larger sound speed by exactly the closing speed, for a separating
    pair it is the larger sound speed."""
    mp.mp.dps = 50
    cfg, s = _pair_state(orc, approach)
    out = orc.rates(cfg, s)
    assert out["nbr_count"].tolist() == [1, 1]
    for i, j in ((0, 1), (1, 0)):
        ref = _two_particle_rates(_mp_state(s, i), _mp_state(s, j), mp.mpf(SUPPORT))
        assert (ref["closing"] > 0) == approach
        for k in ("drho", "dvx", "dvy", "dvz", "dE", "signal"):
            want = float(ref[k])
            assert abs(out[k][i] - want) <= 2e-14 * abs(want) + 1e-300, (i, k, out[k][i], want)
        if not approach:
            ca = float(_pressure_sound(_mp_state(s, 0))[1])
            cb = float(_pressure_sound(_mp_state(s, 1))[1])
            assert out["signal"][i] == max(ca, cb)


def test_two_particle_step_by_hand(orc):
    """One step of fixed dt with non-zero rates: v, E, rho advance by dt times the
    50-digit rates, then the positions by dt times the NEW velocity (symplectic Euler,
    the state renewal of Algorithm 1 as read here); the old-velocity update is far off."""
    mp.mp.dps = 50
    cfg, s = _pair_state(orc, True)
    dt = 0.1
    s1, t1, dtu, cnt = orc.step(cfg, s, t=2.0, dt_in=dt)
    assert dtu == dt and t1 == 2.1 and cnt.tolist() == [1, 1]
    for i, j in ((0, 1), (1, 0)):
        a = _mp_state(s, i)
        ref = _two_particle_rates(a, _mp_state(s, j), mp.mpf(SUPPORT))
        D = mp.mpf(dt)
        v_new = {c: a["v" + c] + D * ref["dv" + c] for c in ("x", "y", "z")}
        want = dict(rho=a["rho"] + D * ref["drho"], E=a["E"] + D * ref["dE"],
                    **{"v" + c: v_new[c] for c in ("x", "y", "z")},
                    **{c: a[c] + D * v_new[c] for c in ("x", "y", "z")})
        for k, v in want.items():
            assert abs(s1[k][i] - float(v)) <= 4e-16 * (1 + abs(float(v))), (i, k)
        # the update with the old velocity differs by dt^2 |dv/dt|, far above rounding
        old = float(a["x"] + D * a["vx"])
        assert abs(s1["x"][i] - old) > 1e3 * 4e-16 * (1 + abs(old))
    assert s1["m"].tolist() == s["m"].tolist()


def _one_particle(orc, x, vx, wall):
    cfg = orc.make_cfg([(0, GAMMA, 0.0)], h=H_SMOOTH, kappa=KAPPA, cfl=0.0, wall=wall)
    one = lambda a: np.array([a], np.float64)
    s = dict(x=one(x), y=one(0.5), z=one(-0.25), vx=one(vx), vy=one(0.3), vz=one(-0.1),
             rho=one(1.0), m=one(1.0), mat=np.zeros(1, np.int32))
    s["E"] = orc.init_energy(cfg, s["rho"], one(1.0), s["vx"], s["vy"], s["vz"], s["mat"])
    return cfg, s


@pytest.mark.parametrize("vw", [0.0, 0.5])
def test_wall_stops_a_particle_by_hand(orc, vw):
    """A particle farther from the piston than the support (no partner, not even its own
    image) crosses the plane within one step: it is reflected off the rigid wall
    (sec. 7.1) in the wall's frame, x -> 2 x_w(t + dt) - x, v_x -> 2 v_w - v_x, keeping its
    specific internal energy; y, z, rho and the other velocity components move ballistically."""
    cfg, s = _one_particle(orc, 4.0, -50.0, wall=(0.0, vw))
    t0, dt = 1.0, 0.1
    s1, t1, _, cnt = orc.step(cfg, s, t=t0, dt_in=dt)
    assert cnt.tolist() == [0]
    xw = vw * (t0 + dt)
    free = 4.0 + dt * -50.0
    assert free < xw
    assert s1["x"][0] == pytest.approx(2 * xw - free, abs=1e-15)
    assert s1["vx"][0] == 2 * vw + 50.0
    assert s1["y"][0] == 0.5 + dt * 0.3 and s1["vy"][0] == 0.3 and s1["rho"][0] == 1.0
    e0 = s["E"][0] - 0.5 * (s["vx"][0] ** 2 + 0.3 ** 2 + 0.1 ** 2)
    e1 = s1["E"][0] - 0.5 * (s1["vx"][0] ** 2 + 0.3 ** 2 + 0.1 ** 2)
    assert e1 == pytest.approx(e0, rel=1e-12)
    # the same particle not reaching the plane moves ballistically
    cfg, s = _one_particle(orc, 8.0, -20.0, wall=(0.0, vw))
    s1, _, _, _ = orc.step(cfg, s, t=t0, dt_in=dt)
    assert s1["x"][0] == 8.0 + dt * -20.0 and s1["vx"][0] == -20.0


@pytest.mark.slow
def test_piston_wall_holds_porous_run(orc):
    """Porous 32^3 sample (30 % voids, radius 5) driven by the piston at v = 2 with the
    recipe's impulsive start: over 100 CFL steps no particle ever lies behind the piston."""
    w = ci.config2(nside=32)
    cfg = orc.cfg_for(w, search=1)
    s = orc.state_from(w, cfg)
    t = 0.0
    x0, vw = w.wall
    for _ in range(100):
        s_new, t, dt, _ = orc.step(cfg, s, t)
        xw = x0 + vw * t
        assert np.all(s_new["x"] >= xw), (t, int(np.sum(s_new["x"] < xw)))
        s = s_new
    # the piston has pushed into the sample: particles near it move with it
    near = s["x"] < x0 + vw * t + 1.0
    assert near.sum() > 0 and np.median(s["vx"][near]) > 1.0


def test_density_limit_bounds_relative_change(orc):
    """dt's density term (reading R8) keeps every particle's relative density change of one
    step at or below the Courant number, with equality at the binding particle, on an open
    cube whose free surface expands (where the term binds)."""
    w = ci.jittered_block(8, 8, 8, seed=3, p=1.0)
    # a uniformly expanding cube, v = 0.5 (r - centre): div v = 1.5
    w.vx, w.vy, w.vz = (0.5 * (c - 4.0) for c in (w.x, w.y, w.z))
    cfg = orc.cfg_for(w, search=1)
    s = orc.state_from(w, cfg)
    r = orc.rates(cfg, s)
    courant = orc.dt(cfg, r["signal"])
    full = orc.dt(cfg, r["signal"], rho=s["rho"], drho=r["drho"])
    assert full < courant  # the density term binds here
    s1, _, dt, _ = orc.step(cfg, s, 0.0)
    assert dt == full
    rel = np.abs(s1["rho"] - s["rho"]) / s["rho"]
    assert rel.max() <= cfg.cfl * (1 + 1e-14)
    assert rel.max() >= cfg.cfl * (1 - 1e-14)


def _wall_pair_cloud():
    w = ci.random_cloud(1200, seed=31, box=7.0, vmax=0.6, n_mat=2)
    w.wall = (1.5, 0.3)
    return w


@pytest.mark.parametrize("mode", ["wall", "pair", "plain"])
def test_rates_sample_equals_full_evaluation(orc, mode):
    """The sampled rate evaluation returns, bit for bit, the full evaluation's values of the
    listed particles (any order, repeats), with the piston wall and in pair-h mode."""
    w = _wall_pair_cloud() if mode == "wall" else ci.random_cloud(1200, seed=32, box=7.0,
                                                                   n_mat=2)
    d = None
    over = {}
    if mode == "pair":
        d = np.random.default_rng(3).uniform(0.8, 1.3, w.n)
        over = dict(h_mode=1, kappa=1.936, cell_size=0.0)
    if mode != "wall":
        w.wall = None
    for search in (0, 1):
        cfg = orc.cfg_for(w, search=search, **over)
        s = orc.state_from(w, cfg)
        full = orc.rates(cfg, s, t=0.7, d=d)
        sample = np.array([5, 0, w.n - 1, 17, 17, 600, 3, 999], np.int64)
        part = orc.rates_sample(cfg, s, sample, t=0.7, d=d)
        for k in ("drho", "dvx", "dvy", "dvz", "dE", "signal", "nbr_count"):
            assert np.array_equal(part[k], full[k][sample]), (search, k)


@pytest.mark.parametrize("D", [1.0, 1.5, 2.2])
@pytest.mark.parametrize("wl", ["cloud", "wall", "behind", "pair"])
def test_cell_list_small_cells_equals_brute_force(orc, wl, D):
    """With mesh cells smaller than the support (reach ceil(H/D) = 2 or 3 cells) the
    cell-list neighbour sets and rates are those of the brute-force search, bit for bit,
    also with the piston wall in front of and inside the particle set."""
    d = None
    over = {}
    if wl == "cloud":
        w = ci.random_cloud(2500, seed=41, box=9.0, n_mat=2)
    elif wl == "pair":
        w = ci.random_cloud(2000, seed=42, box=8.0)
        d = np.random.default_rng(5).uniform(0.7, 1.2, w.n)
        over = dict(h_mode=1, kappa=1.936)
    else:
        w = ci.jittered_block(11, 9, 8, seed=43, v=(-0.2, 0.1, 0.0))
        w.wall = (0.0, 0.4) if wl == "wall" else (6.0, 0.0)
    cb = orc.cfg_for(w, search=0, **over)
    cg = orc.cfg_for(w, search=1, **{**over, "cell_size": D})
    s = orc.state_from(w, cb)
    ob, ib = orc.neighbors(cb, s["x"], s["y"], s["z"], d)
    og, ig = orc.neighbors(cg, s["x"], s["y"], s["z"], d)
    assert np.array_equal(ob, og) and np.array_equal(ib, ig)
    rb = orc.rates(cb, s, t=0.3, d=d)
    rg = orc.rates(cg, s, t=0.3, d=d)
    for k in ("drho", "dvx", "dvy", "dvz", "dE", "signal", "nbr_count"):
        assert np.array_equal(rb[k], rg[k]), k


def test_signal_speed_galilean_invariant(orc):
    """The signal speed depends on velocity differences only: adding u to every velocity
    leaves it unchanged (bit for bit up to the rounding of v_L - v_R)."""
    w = ci.random_cloud(1500, seed=8, box=8.0, n_mat=2, vmax=1.0)
    cfg = orc.cfg_for(w, search=1)
    s = orc.state_from(w, cfg)
    r0 = orc.rates(cfg, s)
    s2 = {k: v.copy() for k, v in s.items()}
    u = (0.7, -1.1, 0.4)
    for c, du in zip(("vx", "vy", "vz"), u):
        s2[c] = s[c] + du
    s2["E"] = orc.init_energy(cfg, s["rho"], np.ascontiguousarray(w.p), s2["vx"], s2["vy"],
                              s2["vz"], s["mat"])
    r1 = orc.rates(cfg, s2)
    assert np.abs(r1["signal"] - r0["signal"]).max() <= 1e-13 * r0["signal"].max()
    # and it exceeds the sound speed somewhere (pairs are closing)
    P, c, _ = orc.eos(cfg, s)
    assert np.any(r0["signal"] > c * (1 + 1e-3))
