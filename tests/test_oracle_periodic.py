"""Pins of the oracle's periodic boundaries (the PBC of the paper's static-plate and ejecta
tests, secs. 6 and 7.1): partners are the periodic images of the particles, with the
displacement (x_j - x_i) - k L along each periodic axis (k in {-1, 0, 1}); the step wraps
positions back into the box.

The pins: a perfect periodic lattice has no boundary (every particle has the interior count
and zero rates), the neighbour sets equal a numpy brute force over the images, the cell list
equals the brute force, the relation is symmetric, a closed periodic box conserves momentum
and energy, the rates do not depend on where the box's origin cuts the lattice, and a
particle leaving through one face re-enters through the other.
"""
import json
import os

import numpy as np
import pytest

import csph_inputs as ci

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _images_brute_force(w, H):
    """{i: sorted j} with |(r_j - r_i) - k L| < H for some k (k_a = 0 off the periodic axes),
    (j, k) != (i, 0), in numpy FP64 with the same operation order."""
    P = np.stack([w.x, w.y, w.z], 1)
    L = np.array([(w.box[1][a] - w.box[0][a]) if (w.periodic >> a) & 1 else 0.0
                  for a in range(3)])
    ks = [(kx, ky, kz) for kz in (-1, 0, 1) for ky in (-1, 0, 1) for kx in (-1, 0, 1)
          if all(k == 0 or L[a] > 0 for a, k in enumerate((kx, ky, kz)))]
    out = {}
    for i in range(w.n):
        d0 = P - P[i]
        hits = set()
        for k in ks:
            d = d0.copy()
            for a in range(3):
                if k[a]:
                    d[:, a] = d[:, a] - k[a] * L[a]
            r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
            for j in np.nonzero(r2 < H * H)[0]:
                if j == i and k == (0, 0, 0):
                    continue
                hits.add(int(j))
        out[i] = sorted(hits)
    return out


def test_periodic_lattice_has_no_boundary(orc):
    """A perfect lattice filling a periodic 10^3 box: every particle sees the interior count
    of the unit lattice (92 within support 3, from the golden file) and, in a uniform state,
    zero rates; the same lattice with open boundaries has 1 000 - 216 surface particles
    with fewer partners and non-zero rates."""
    gold = json.load(open(os.path.join(GOLD, "lattice_counts.json")))
    want = [c["interior_count"] for c in gold["cases"] if c["h"] == 1.5][0]
    w = ci.periodic_block(10, 10, 10, seed=0, periodic=7, amp=0.0)
    cfg = orc.cfg_for(w, search=1)
    s = orc.state_from(w, cfg)
    r = orc.rates(cfg, s)
    assert r["nbr_count"].tolist() == [want] * w.n
    for k in ("drho", "dvx", "dvy", "dvz", "dE"):
        assert np.abs(r[k]).max() < 1e-14, k
    w.periodic = 0
    r_open = orc.rates(orc.cfg_for(w, search=1), s)
    assert (r_open["nbr_count"] < want).sum() == 1000 - 216
    assert np.abs(r_open["dvx"]).max() > 1e-3


@pytest.mark.parametrize("mask", [7, 1, 6])
def test_periodic_neighbours_equal_image_brute_force(orc, mask):
    w = ci.periodic_block(9, 8, 7, seed=3, periodic=mask, amp=0.2)
    cfg = orc.cfg_for(w, search=0)
    off, idx = orc.neighbors(cfg, w.x, w.y, w.z)
    ref = _images_brute_force(w, w.kappa * w.h)
    for i in range(w.n):
        assert idx[off[i]:off[i + 1]].tolist() == ref[i], i
    # the relation is symmetric (the displacement is exactly antisymmetric)
    pairs = {(i, int(j)) for i in range(w.n) for j in idx[off[i]:off[i + 1]]}
    assert all((j, i) in pairs for i, j in pairs)


@pytest.mark.parametrize("D", [0.0, 1.0, 2.2])
@pytest.mark.parametrize("case", ["xyz", "yz+wall", "pair-h"])
def test_periodic_cell_list_equals_brute_force(orc, case, D):
    d = None
    over = {}
    if case == "xyz":
        w = ci.periodic_block(9, 8, 8, seed=4, periodic=7, amp=0.2, v=(0.1, -0.2, 0.3))
    elif case == "yz+wall":
        w = ci.periodic_block(12, 8, 7, seed=5, periodic=6, amp=0.2, v=(-0.3, 0.1, 0.0))
        w.wall = (0.25, 0.5)
    else:
        w = ci.periodic_block(8, 8, 8, seed=6, periodic=7, amp=0.2)
        d = np.random.default_rng(2).uniform(0.8, 1.2, w.n)
        over = dict(h_mode=1, kappa=1.936)
    cb = orc.cfg_for(w, search=0, **over)
    cg = orc.cfg_for(w, search=1, **{**over, "cell_size": D})
    s = orc.state_from(w, cb)
    ob, ib = orc.neighbors(cb, s["x"], s["y"], s["z"], d)
    og, ig = orc.neighbors(cg, s["x"], s["y"], s["z"], d)
    assert np.array_equal(ob, og) and np.array_equal(ib, ig)
    rb = orc.rates(cb, s, t=0.2, d=d)
    rg = orc.rates(cg, s, t=0.2, d=d)
    for k in ("drho", "dvx", "dvy", "dvz", "dE", "signal", "nbr_count"):
        assert np.array_equal(rb[k], rg[k]), k


def test_closed_periodic_box_conserves(orc):
    """No boundary, no wall: the pair terms cancel, sum m dv/dt = sum m dE/dt = 0."""
    w = ci.periodic_block(9, 9, 9, seed=8, periodic=7, amp=0.3)
    rng = np.random.default_rng(8)
    w.vx, w.vy, w.vz = (rng.uniform(-0.5, 0.5, w.n) for _ in range(3))
    w.p = rng.uniform(0.5, 2.0, w.n)
    cfg = orc.cfg_for(w, search=1)
    s = orc.state_from(w, cfg)
    r = orc.rates(cfg, s)
    for k in ("dvx", "dvy", "dvz", "dE"):
        terms = s["m"] * r[k]
        assert abs(orc.exact_sum(terms)) < 1e-13 * np.abs(terms).sum(), k
    s1, t1, dt, _ = orc.step(cfg, s, 0.0)
    tot0, tot1 = orc.totals(s), orc.totals(s1)
    assert tot1[0] == tot0[0]
    for k in (1, 2, 3, 4):
        assert abs(tot1[k] - tot0[k]) < 1e-13 * (np.abs(s["m"]).sum() * (1 + np.abs(s["E"]).max()))


def test_periodic_rates_independent_of_the_cut(orc):
    """Shifting every particle by s along the periodic x axis (wrapped into the box) moves
    the box's cut through the material: the rates of each particle stay the same."""
    w = ci.periodic_block(10, 8, 8, seed=9, periodic=7, amp=0.3)
    rng = np.random.default_rng(9)
    w.vx, w.vy, w.vz = (rng.uniform(-0.4, 0.4, w.n) for _ in range(3))
    w.p = rng.uniform(0.5, 2.0, w.n)
    cfg = orc.cfg_for(w, search=1)
    s = orc.state_from(w, cfg)
    r = orc.rates(cfg, s)
    s2 = {k: v.copy() for k, v in s.items()}
    x = s["x"] + 3.7
    s2["x"] = np.where(x >= 10.0, x - 10.0, x)
    r2 = orc.rates(cfg, s2)
    assert np.array_equal(r["nbr_count"], r2["nbr_count"])
    for k in ("drho", "dvx", "dvy", "dvz", "dE"):
        assert np.abs(r2[k] - r[k]).max() <= 1e-12 * np.abs(r[k]).max(), k


def test_step_wraps_through_the_faces(orc):
    """Two isolated particles moving out through opposite faces re-enter through the other
    face: x + dt v - L and x + dt v + L."""
    L = 20.0
    s = dict(x=np.array([19.9, 0.05]), y=np.array([10.0, 5.0]), z=np.array([10.0, 5.0]),
             vx=np.array([1.0, -1.0]), vy=np.zeros(2), vz=np.array([0.0, 0.5]),
             rho=np.ones(2), m=np.ones(2), mat=np.zeros(2, np.int32))
    cfg = orc.make_cfg([(0, 1.4, 0.0)], cfl=0.0, periodic=7,
                       box=((0.0, 0.0, 0.0), (L, L, L)))
    s["E"] = orc.init_energy(cfg, s["rho"], np.ones(2), s["vx"], s["vy"], s["vz"], s["mat"])
    s1, t, dt, cnt = orc.step(cfg, s, 0.0, dt_in=0.25)
    assert cnt.tolist() == [0, 0]
    assert s1["x"].tolist() == [(19.9 + 0.25) - L, (0.05 - 0.25) + L]
    assert s1["z"].tolist() == [10.0, 5.0 + 0.125]
    assert np.array_equal(s1["vx"], s["vx"]) and np.array_equal(s1["E"], s["E"])


@pytest.mark.parametrize("mask", [0, 6])
def test_wall_mirror_partners_equal_explicit_reflected_particles(orc, mask):
    """The rigid wall's mirror partners (sec. 7.1, reading: the piston reflects the particles
    within the support of it) are the particles reflected in the piston plane, x -> 2 x_w - x,
    v_x -> 2 v_w - v_x, with their density, mass and pressure: adding those reflected
    particles as real ones to a wall-free system (periodic along y and z when mask = 6, where
    their periodic images are partners too) gives the real particles the same rates."""
    w = ci.periodic_block(10, 8, 7, seed=11, periodic=mask, amp=0.25)
    rng = np.random.default_rng(11)
    w.vx, w.vy, w.vz = (rng.uniform(-0.5, 0.5, w.n) for _ in range(3))
    w.p = rng.uniform(0.5, 2.0, w.n)
    x0, vw, t = -0.6, 0.7, 0.5
    w.wall = (x0, vw)
    xw = x0 + vw * t
    assert xw < w.x.min() and (w.x < xw + w.kappa * w.h).sum() > 100
    cfg = orc.cfg_for(w, search=1)
    s = orc.state_from(w, cfg)
    r = orc.rates(cfg, s, t=t)
    g = {k: np.concatenate([np.asarray(getattr(w, k), np.float64)] * 2)
         for k in ("y", "z", "vy", "vz", "rho", "m", "p")}
    g["x"] = np.concatenate([w.x, 2.0 * xw - w.x])
    g["vx"] = np.concatenate([w.vx, 2.0 * vw - w.vx])
    g["mat"] = np.zeros(2 * w.n, np.int32)
    box = ((2.0 * xw - 10.0, 0.0, 0.0), (10.0, 8.0, 7.0))
    ce = orc.make_cfg(w.eos, h=w.h, kappa=w.kappa, search=1, periodic=mask, box=box)
    se = {k: g[k] for k in ("x", "y", "z", "vx", "vy", "vz", "rho", "m", "mat")}
    se["E"] = orc.init_energy(ce, g["rho"], g["p"], g["vx"], g["vy"], g["vz"], g["mat"])
    re = orc.rates(ce, se)
    for k in ("drho", "dvx", "dvy", "dvz", "dE"):
        scale = np.abs(r[k]).max()
        assert np.abs(re[k][:w.n] - r[k]).max() <= 1e-12 * scale, k
    assert np.allclose(re["signal"][:w.n], r["signal"], rtol=1e-14, atol=0)
