"""The library's Sod tube against the oracle's (and so against the exact Riemann solution the
oracle is checked on): 160 x 7 x 7 particles, periodic across, the CFL rule, to t ~ 12, particle
order kept; fixed h (57 steps) in FP64 and in mixed precision, and the paper's pair-h mode
(kappa = 1.936) with the sizes d = (m/rho)^(1/3) formed on the host before every step, as a
caller does, in FP64, and the two-stage Runge-Kutta step in FP64."""
import numpy as np
import pytest
import torch

import csph_inputs as ci
import oracle as O
import paper_1805_05128_amd as P
from helpers import to_np

pytestmark = pytest.mark.gpu

DEV = "cuda"
T_END = 12.0


def _tube():
    w = ci.periodic_block(160, 7, 7, seed=5, periodic=6)
    left = w.x < 80.0
    w.rho = np.where(left, 1.0, 0.125)
    w.p = np.where(left, 1.0, 0.1)
    w.m = w.rho.copy()
    return w


@pytest.fixture(scope="module")
def oracle_run():
    w = _tube()
    cfg = O.cfg_for(w, search=1)
    s = O.state_from(w, cfg)
    t, dts = 0.0, []
    while t < T_END:
        s, t, dt, _ = O.step(cfg, s, t)
        dts.append(dt)
    return w, s, t, dts


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("mixed", 2e-3)])
def test_sod_tube_matches_the_oracle(oracle_run, prec, tol):
    w, s_ref, t_ref, dts = oracle_run
    print(f"[case] sod tube {prec} n={w.n} steps={len(dts)}", flush=True)
    params = P.Params.from_workload(w, precision=prec, reorder=False)
    g = P.state_from_workload(w, params, DEV)
    sc = P.StepScalars(DEV)
    for _ in range(len(dts)):
        P.csph_step(g, params, sc, s_out=g, totals=False)
    torch.cuda.synchronize()
    # the same number of CFL steps lands on the same time (FP64: to rounding)
    assert abs(to_np(sc.t)[0] - t_ref) <= (1e-12 if prec == "fp64" else 1e-3) * t_ref
    for k, scale in (("x", 1.0), ("vx", 1.0), ("rho", 1.0), ("E", 1.0)):
        err = np.abs(to_np(g[k]) - s_ref[k]).max()
        assert err <= tol * scale, (k, err)


def test_sod_tube_pair_h_matches_the_oracle():
    w = _tube()
    cfg = O.cfg_for(w, search=1, h_mode=1, kappa=1.936)
    s = O.state_from(w, cfg)
    t, nsteps = 0.0, 0
    while t < T_END:
        s, t, _, _ = O.step(cfg, s, t, d=np.cbrt(s["m"] / s["rho"]))
        nsteps += 1
    print(f"[case] sod tube pair-h n={w.n} steps={nsteps}", flush=True)
    params = P.Params.from_workload(w, reorder=False, h_mode="pair", kappa=1.936, cell_size=0.0)
    g = P.state_from_workload(w, params, DEV)
    m = to_np(g["m"])
    sc = P.StepScalars(DEV)
    for _ in range(nsteps):
        g.d = torch.as_tensor(np.cbrt(m / to_np(g["rho"])), device=DEV)
        P.csph_step(g, params, sc, s_out=g, totals=False)
    torch.cuda.synchronize()
    assert abs(to_np(sc.t)[0] - t) <= 1e-12 * t
    for k in ("x", "vx", "rho", "E"):
        err = np.abs(to_np(g[k]) - s[k]).max()
        assert err <= 1e-9, (k, err)


def test_sod_tube_rk2_matches_the_oracle():
    w = _tube()
    cfg = O.cfg_for(w, search=1, integrator=1)
    s = O.state_from(w, cfg)
    t, nsteps = 0.0, 0
    while t < T_END:
        s, t, _, _ = O.step(cfg, s, t)
        nsteps += 1
    print(f"[case] sod tube rk2 n={w.n} steps={nsteps}", flush=True)
    params = P.Params.from_workload(w, reorder=False, integrator="rk2")
    g = P.state_from_workload(w, params, DEV)
    sc = P.StepScalars(DEV)
    for _ in range(nsteps):
        P.csph_step(g, params, sc, s_out=g, totals=False)
    torch.cuda.synchronize()
    assert abs(to_np(sc.t)[0] - t) <= 1e-12 * t
    for k in ("x", "vx", "rho", "E"):
        err = np.abs(to_np(g[k]) - s[k]).max()
        assert err <= 1e-9, (k, err)
