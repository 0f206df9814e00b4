"""GPU parity of the periodic boundaries (the PBC of the paper's plate tests, secs. 6 and 7.1)
against the oracle: neighbour sets bit-exact, rates in both precisions, the step with its wrap
through the faces, the piston wall with periodic sides, and the errors the library raises.
"""
import numpy as np
import pytest
import torch

import csph_inputs as ci
import oracle as O
import paper_1805_05128_amd as P
from helpers import field_relerr, rates_np, to_np

pytestmark = pytest.mark.gpu

DEV = "cuda"
FP64_TOL = 1e-12
MIXED_TOL = 2e-5


def _print_case(name, w):
    print(f"[case] {name} n={w.n} periodic={w.periodic}", flush=True)


def _stirred(w, seed, vmax=0.5):
    """Random velocities and pressures (every pair term non-zero)."""
    rng = np.random.default_rng(seed)
    w.vx, w.vy, w.vz = (rng.uniform(-vmax, vmax, w.n) for _ in range(3))
    w.p = rng.uniform(0.5, 2.0, w.n)
    return w


def xyz_box():
    return _stirred(ci.periodic_block(11, 9, 13, seed=1, periodic=7, amp=0.3), 1)


def x_only():
    return _stirred(ci.periodic_block(12, 8, 9, seed=2, periodic=1, amp=0.3), 2)


def yz_wall():
    """The plate geometry: piston wall along x, periodic across it (y, z)."""
    w = _stirred(ci.periodic_block(14, 9, 10, seed=3, periodic=6, amp=0.3), 3)
    w.wall = (0.1, 0.6)
    return w


def lattice():
    """Perfect lattice filling the box: every pair distance a lattice distance, some exactly
    the support (ties the strict test must reject)."""
    return ci.periodic_block(10, 10, 10, seed=0, periodic=7, amp=0.0)


def small_cells():
    w = _stirred(ci.periodic_block(9, 10, 8, seed=4, periodic=5, amp=0.3), 4)
    w.cell_size = 1.1
    return w


CASES = {"xyz": xyz_box, "x": x_only, "yz+wall": yz_wall, "lattice": lattice,
         "small-cells": small_cells}


def _cfg(w, **over):
    return O.cfg_for(w, search=1, **over)


@pytest.mark.parametrize("case", list(CASES))
def test_periodic_neighbors_bitexact(case):
    w = CASES[case]()
    _print_case(case, w)
    params = P.Params.from_workload(w)
    g = P.state_from_workload(w, params, DEV)
    off, idx = P.csph_neighbors(g, params)
    torch.cuda.synchronize()
    ro, ri = O.neighbors(_cfg(w), w.x, w.y, w.z)
    assert np.array_equal(to_np(off), ro)
    assert np.array_equal(to_np(idx), ri)
    if case == "lattice":
        assert np.all(np.diff(ro) == 92)


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
@pytest.mark.parametrize("case", list(CASES))
def test_periodic_rates(case, prec, tol):
    w = CASES[case]()
    _print_case(f"{case} {prec}", w)
    params = P.Params.from_workload(w, precision=prec)
    g = P.state_from_workload(w, params, DEV)
    got = rates_np(P.csph_rates(g, params, t=0.3))
    torch.cuda.synchronize()
    ref = O.rates(_cfg(w), O.state_from(w, _cfg(w)), t=0.3)
    assert np.array_equal(got["nbr_count"].astype(np.int64), ref["nbr_count"])
    if case == "lattice":  # no boundary: zero rates
        for k in ("drho", "dvx", "dvy", "dvz", "dE"):
            assert np.abs(got[k]).max() <= (1e-13 if prec == "fp64" else 1e-6), k
        return
    err = field_relerr(got, ref)
    print(prec, "relerr", err)
    assert max(err.values()) <= tol, err
    stol = 1e-13 if prec == "fp64" else 1e-5
    assert np.abs(got["signal"] - ref["signal"]).max() <= stol * ref["signal"].max()


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_periodic_rates_pair_h(prec, tol):
    w = _stirred(ci.periodic_block(9, 9, 9, seed=6, periodic=7, amp=0.25), 6)
    d = np.random.default_rng(6).uniform(0.8, 1.2, w.n)
    _print_case(f"pair-h {prec}", w)
    params = P.Params.from_workload(w, precision=prec, h_mode="pair", kappa=1.936, cell_size=0.0)
    g = P.state_from_workload(w, params, DEV)
    g.d = torch.as_tensor(d, dtype=torch.float64, device=DEV)
    got = rates_np(P.csph_rates(g, params))
    off, idx = P.csph_neighbors(g, params)
    torch.cuda.synchronize()
    cfg = _cfg(w, h_mode=1, kappa=1.936)
    ref = O.rates(cfg, O.state_from(w, cfg), d=d)
    ro, ri = O.neighbors(cfg, w.x, w.y, w.z, d)
    assert np.array_equal(to_np(off), ro) and np.array_equal(to_np(idx), ri)
    assert np.array_equal(got["nbr_count"].astype(np.int64), ref["nbr_count"])
    err = field_relerr(got, ref)
    assert max(err.values()) <= tol, err


def _fast_box(seed, periodic=7):
    """Bulk motion (dt ~ 0.2) that carries the particles within ~0.5 of a face through it in
    one step."""
    w = _stirred(ci.periodic_block(10, 9, 11, seed=seed, periodic=periodic, amp=0.3), seed,
                 vmax=0.3)
    w.vx = w.vx + 3.0
    w.vy = w.vy - 2.5
    w.vz = w.vz + 2.5
    return w


@pytest.mark.parametrize("reorder", [False, True])
@pytest.mark.parametrize("case", ["fast-xyz", "fast-xz", "yz+wall"])
def test_periodic_step_fp64(case, reorder):
    """fast-xz: x periodic with y open, which the library hands to the kernels as their x."""
    w = {"fast-xyz": lambda: _fast_box(8), "fast-xz": lambda: _fast_box(8, periodic=5),
         "yz+wall": yz_wall}[case]()
    _print_case(f"step {case} reorder={reorder}", w)
    params = P.Params.from_workload(w, reorder=reorder)
    g = P.state_from_workload(w, params, DEV)
    sc = P.StepScalars(DEV, t0=0.125)
    cnt = torch.empty(w.n, dtype=torch.int32, device=DEV)
    out = P.csph_step(g, params, sc, nbr_count=cnt)
    torch.cuda.synchronize()
    cfg = _cfg(w)
    s0 = O.state_from(w, cfg)
    s1, t1, dt, ncount = O.step(cfg, s0, t=0.125)
    got = out.numpy()
    ids = got["id"]
    assert np.array_equal(np.sort(ids), np.arange(w.n))
    assert abs(to_np(sc.dt)[0] - dt) <= 1e-15 * dt
    if case.startswith("fast"):  # some particles crossed each periodic face pair
        for a, (k, L) in enumerate((("x", 10.0), ("y", 9.0), ("z", 11.0))):
            if (w.periodic >> a) & 1:
                assert np.sum(np.abs(s1[k] - s0[k]) > L / 2) > 10, k
    for k in ("x", "y", "z", "vx", "vy", "vz", "rho", "E"):
        a, b = got[k], s1[k][ids]
        inc = b - s0[k][ids]
        if k in ("x", "y", "z"):  # the wrapped increment is the unwrapped one
            inc = np.where(np.abs(inc) > 4.0, 0.0, inc)
        den = max(np.abs(inc).max(), 1e-300)
        assert np.abs(a - b).max() <= FP64_TOL * den + 4 * np.finfo(float).eps * np.abs(b).max(), k
    assert np.array_equal(to_np(cnt).astype(np.int64), ncount[ids])
    lo, hi = np.array(w.box[0]), np.array(w.box[1])
    for a, k in enumerate(("x", "y", "z")):
        if (w.periodic >> a) & 1:
            assert got[k].min() >= lo[a] and got[k].max() < hi[a], k


@pytest.mark.parametrize("mask", [7, 5])
def test_periodic_step_mixed_and_voronoi(mask):
    """Mixed-precision step with the fused Voronoi ownership of the wrapped positions (mask 5:
    the kernels take the caller's y as x)."""
    w = _fast_box(9, periodic=mask)
    params = P.Params.from_workload(w, precision="mixed", reorder=True)
    g = P.state_from_workload(w, params, DEV)
    sites = torch.as_tensor(ci.voronoi_sites(37, seed=9, box=(10.0, 9.0, 11.0)), device=DEV)
    owner = torch.empty(w.n, dtype=torch.int32, device=DEV)
    sp = torch.empty(37, dtype=torch.int64, device=DEV)
    spairs = torch.empty(37, dtype=torch.int64, device=DEV)
    sc = P.StepScalars(DEV)
    cnt = torch.empty(w.n, dtype=torch.int32, device=DEV)
    out = P.csph_step_voronoi(g, params, sc, sites, owner, sp, spairs, nbr_count=cnt)
    torch.cuda.synchronize()
    got = out.numpy()
    ids = got["id"]
    cfg = _cfg(w)
    s0 = O.state_from(w, cfg)
    dt = float(to_np(sc.dt)[0])
    s1, _, _, ncount = O.step(cfg, s0, t=0.0, dt_in=dt)
    assert np.array_equal(to_np(cnt).astype(np.int64), ncount[ids])
    for k in ("x", "y", "z"):  # positions within the mixed tolerance of the FP64 step
        d = np.abs(got[k] - s1[k][ids])
        d = np.minimum(d, np.abs(d - {"x": 10.0, "y": 9.0, "z": 11.0}[k]))
        assert d.max() <= 1e-6, k
    ro, rsp, rspairs = O.voronoi(got["x"], got["y"], got["z"], to_np(sites),
                                 to_np(cnt).astype(np.int64))
    assert np.array_equal(to_np(owner), ro)
    assert np.array_equal(to_np(sp), rsp) and np.array_equal(to_np(spairs), rspairs)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_periodic_box_over_steps(prec):
    """30 CFL steps of a stirred periodic box with bulk motion: the positions stay in the box,
    mass is exact and momentum and energy stay at their start values (no boundary, no wall)."""
    w = _fast_box(10)
    params = P.Params.from_workload(w, precision=prec, reorder=True)
    g = P.state_from_workload(w, params, DEV)
    sc = P.StepScalars(DEV)
    tot = []
    for _ in range(30):
        g = P.csph_step(g, params, sc)
        tot.append(to_np(sc.totals).reshape(5, 2).sum(1))
    torch.cuda.synchronize()
    got = g.numpy()
    for a, (k, L) in enumerate((("x", 10.0), ("y", 9.0), ("z", 11.0))):
        assert got[k].min() >= 0.0 and got[k].max() < L, k
    tot = np.array(tot)
    m = np.abs(got["m"]).sum()
    assert np.all(tot[:, 0] == tot[0, 0])
    drift = np.abs(tot - tot[0]).max(0)
    scale = m * (1.0 + np.abs(got["E"]).max())
    tol = 1e-11 if prec == "fp64" else 1e-4
    assert drift[1:].max() <= tol * scale, drift


def test_periodic_errors():
    w = xyz_box()
    params = P.Params.from_workload(w)
    g = P.state_from_workload(w, params, DEV)
    # a period not above twice the support (H = 3)
    small = P.Params.from_workload(w, box=((0.0, 0.0, 0.0), (11.0, 9.0, 6.0)))
    with pytest.raises(P.CsphError, match="period"):
        P.csph_rates(g, small)
    # positions outside the box
    shifted = P.Params.from_workload(w, box=((0.5, 0.0, 0.0), (11.5, 9.0, 13.0)))
    with pytest.raises(P.CsphError, match="outside"):
        P.csph_rates(g, shifted)
    with pytest.raises(P.CsphError, match="outside"):
        P.csph_step(g, shifted, P.StepScalars(DEV))
    # the wall's axis cannot be periodic
    with pytest.raises(P.CsphError, match="wall"):
        P.csph_rates(g, P.Params.from_workload(w, wall=(-1.0, 0.0)), t=0.0)
    torch.cuda.synchronize()
