"""GPU parity of the two-stage Runge-Kutta step (csph_params.integrator = CSPH_INT_RK2)
against the oracle's: FP64 within 1e-12 of each field's increment, the mixed-precision step
within the FP32 rate tolerance, the first stage's neighbour counts bit-exact, with the piston,
periodic boundaries, pair-h mode, both output orders, and over a run of steps.
"""
import math

import numpy as np
import pytest
import torch

import csph_inputs as ci
import oracle as O
import paper_1805_05128_amd as P
from helpers import to_np
from test_gpu_parity import _check_totals, behind_wall_block, cold_cloud, wall_block

pytestmark = pytest.mark.gpu

DEV = "cuda"
FP64_TOL = 1e-12


def _periodic_fast():
    w = ci.periodic_block(10, 9, 11, seed=31, periodic=7, amp=0.3)
    rng = np.random.default_rng(31)
    w.vx, w.vy, w.vz = (rng.uniform(-0.3, 0.3, w.n) for _ in range(3))
    w.vx = w.vx + 3.0
    w.vy = w.vy - 2.5
    w.p = rng.uniform(0.5, 2.0, w.n)
    return w


def _yz_wall():
    w = ci.periodic_block(14, 9, 10, seed=32, periodic=6, amp=0.3)
    rng = np.random.default_rng(32)
    w.vx, w.vy, w.vz = (rng.uniform(-0.5, 0.5, w.n) for _ in range(3))
    w.p = rng.uniform(0.5, 2.0, w.n)
    w.wall = (0.1, 0.6)
    return w


CASES = {"sod16": ci.config0, "wall": wall_block, "behind": behind_wall_block,
         "cold": cold_cloud, "periodic": _periodic_fast, "yz+wall": _yz_wall}


def _unwrap_inc(k, inc):
    # a wrapped position's increment is the unwrapped one plus or minus a period
    return np.where(np.abs(inc) > 4.0, 0.0, inc) if k in ("x", "y", "z") else inc


@pytest.mark.parametrize("reorder", [False, True])
@pytest.mark.parametrize("case", list(CASES))
def test_rk2_step_fp64(case, reorder):
    w = CASES[case]()
    print(f"[case] rk2 {case} reorder={reorder} n={w.n}", flush=True)
    params = P.Params.from_workload(w, reorder=reorder, integrator="rk2")
    g = P.state_from_workload(w, params, DEV)
    sc = P.StepScalars(DEV, t0=0.125)
    cnt = torch.empty(w.n, dtype=torch.int32, device=DEV)
    out = P.csph_step(g, params, sc, nbr_count=cnt)
    torch.cuda.synchronize()
    cfg = O.cfg_for(w, search=1, integrator=1)
    s0 = O.state_from(w, cfg)
    s1, t1, dt, ncount = O.step(cfg, s0, t=0.125)
    got = out.numpy()
    ids = got["id"]
    if not reorder:
        assert np.array_equal(ids, np.arange(w.n))
    assert np.array_equal(np.sort(ids), np.arange(w.n))
    assert abs(to_np(sc.dt)[0] - dt) <= 1e-15 * dt
    assert abs(to_np(sc.t)[0] - t1) <= 1e-15 * t1
    for k in ("x", "y", "z", "vx", "vy", "vz", "rho", "E"):
        a, b = got[k], s1[k][ids]
        den = max(np.abs(_unwrap_inc(k, b - s0[k][ids])).max(), 1e-300)
        assert np.abs(a - b).max() <= FP64_TOL * den + 4 * np.finfo(float).eps * np.abs(b).max(), k
    assert np.array_equal(got["m"], s0["m"][ids])
    assert np.array_equal(to_np(cnt).astype(np.int64), ncount[ids])
    _check_totals(to_np(sc.totals), got)


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("mixed", 5e-5)])
def test_rk2_step_pair_h(prec, tol):
    w = ci.periodic_block(9, 9, 9, seed=33, periodic=7, amp=0.25)
    rng = np.random.default_rng(33)
    w.vx, w.vy, w.vz = (rng.uniform(-0.5, 0.5, w.n) for _ in range(3))
    w.p = rng.uniform(0.5, 2.0, w.n)
    d = rng.uniform(0.8, 1.2, w.n)
    params = P.Params.from_workload(w, precision=prec, h_mode="pair", kappa=1.936,
                                    cell_size=0.0, reorder=True, integrator="rk2")
    g = P.state_from_workload(w, params, DEV)
    g.d = torch.as_tensor(d, dtype=torch.float64, device=DEV)
    sc = P.StepScalars(DEV)
    out = P.csph_step(g, params, sc)
    torch.cuda.synchronize()
    got = out.numpy()
    ids = got["id"]
    assert np.array_equal(got["d"], d[ids])
    cfg = O.cfg_for(w, search=1, h_mode=1, kappa=1.936, integrator=1)
    s0 = O.state_from(w, cfg)
    dt = float(to_np(sc.dt)[0])
    s1, _, dto, _ = O.step(cfg, s0, t=0.0, dt_in=dt, d=d)
    if prec == "fp64":
        assert abs(dt - O.step(O.cfg_for(w, search=1, h_mode=1, kappa=1.936, integrator=1), s0,
                               t=0.0, d=d)[2]) <= 1e-15 * dt
    for k in ("x", "y", "z", "vx", "vy", "vz", "rho", "E"):
        inc = _unwrap_inc(k, s1[k][ids] - s0[k][ids])
        err = np.abs(got[k] - s1[k][ids])
        if k in ("x", "y", "z"):
            err = np.minimum(err, np.abs(err - 9.0))
        assert err.max() <= tol * np.abs(inc).max() + 4 * np.finfo(float).eps * 9.0, k


def test_rk2_mixed_within_tolerance():
    """Mixed precision: both evaluations' pair arithmetic in FP32; the step's increments stay
    within the FP32 rate tolerance of the FP64 oracle step (same dt)."""
    w = ci.config0()
    params = P.Params.from_workload(w, precision="mixed", reorder=False, integrator="rk2")
    g = P.state_from_workload(w, params, DEV)
    s0 = {k: to_np(v).copy() for k, v in g.t.items()}
    sc = P.StepScalars(DEV)
    P.csph_step(g, params, sc)
    dt = float(to_np(sc.dt)[0])
    got = g.numpy()
    cfg = O.cfg_for(w, search=1, integrator=1)
    s1, _, _, _ = O.step(cfg, O.state_from(w, cfg), t=0.0, dt_in=dt)
    for k in ("x", "y", "z", "vx", "vy", "vz", "rho", "E"):
        inc = s1[k] - s0[k]
        assert np.abs(got[k] - s1[k]).max() <= 5e-5 * np.abs(inc).max() + 1e-15, k


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_rk2_piston_run(prec):
    """Porous 24^3 sample with the piston: 10 RK2 CFL steps, no particle behind the piston,
    mass exact; the FP64 run follows the oracle's RK2 steps."""
    w = ci.config2(nside=24)
    params = P.Params.from_workload(w, precision=prec, reorder=True, integrator="rk2")
    g = P.state_from_workload(w, params, DEV)
    sc = P.StepScalars(DEV)
    cfg = O.cfg_for(w, search=1, integrator=1)
    s = O.state_from(w, cfg)
    t = 0.0
    x0, vw = w.wall
    for step in range(10):
        g = P.csph_step(g, params, sc)
        torch.cuda.synchronize()
        got = g.numpy()
        tg = float(to_np(sc.t)[0])
        assert np.all(got["x"] >= x0 + vw * tg), step
        if prec == "fp64":
            s, t, _, _ = O.step(cfg, s, t)
            assert abs(tg - t) <= 1e-13 * t
            ids = got["id"]
            for k in ("x", "vx", "rho", "E"):
                assert np.abs(got[k] - s[k][ids]).max() <= 1e-10 * (1 + np.abs(s[k]).max()), (step, k)
    m = to_np(sc.totals).reshape(5, 2).sum(1)[0]
    assert math.isclose(m, float(np.sum(w.m)), rel_tol=1e-15)


def test_rk2_refused_by_the_voronoi_step():
    w = ci.config0()
    params = P.Params.from_workload(w, integrator="rk2")
    g = P.state_from_workload(w, params, DEV)
    sites = torch.as_tensor(ci.voronoi_sites(8, seed=1, box=(16.0, 16.0, 16.0)), device=DEV)
    owner = torch.empty(w.n, dtype=torch.int32, device=DEV)
    sp = torch.empty(8, dtype=torch.int64, device=DEV)
    with pytest.raises(P.CsphError, match="Euler"):
        P.csph_step_voronoi(g, params, P.StepScalars(DEV), sites, owner, sp)
    torch.cuda.synchronize()
