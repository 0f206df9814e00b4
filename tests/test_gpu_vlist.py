"""GPU Verlet lists (csph_vlist_build, csph_step_vlist, VerletRun) against
the oracle: the lists are exactly the partners within the horizon
(1 + beta) H (mirror partners included), and runs of list-driven steps
follow the oracle's per-step neighbour search step by step: identical
neighbour counts and time steps, states within tolerance."""
import numpy as np
import pytest
import torch

import csph_inputs as ci
import oracle as O
import paper_1805_05128_amd as P
from helpers import to_np

pytestmark = pytest.mark.gpu
DEV = "cuda"


def wall_block(seed=5):
    w = ci.jittered_block(12, 10, 9, seed=seed, v=(-0.2, 0.1, 0.05))
    w.wall = (0.0, 0.4)
    return w


def behind_block(seed=7):
    """The wall inside the block: particles on both sides of it, some farther behind it
    than the horizon (their mirror partners lie around their image)."""
    w = ci.jittered_block(12, 10, 9, seed=seed, v=(-0.2, 0.1, 0.05))
    w.wall = (5.5, 0.5)
    return w


def moving_cloud(seed=9):
    """Random cloud with large random velocities: the displacement bound forces rebuilds
    before n_upd steps."""
    w = ci.random_cloud(2500, seed=seed, box=11.0, vmax=1.5)
    return w


def slab_cloud(seed=21):
    w = ci.random_cloud(2600, seed=seed, box=8.0, vmax=0.5)
    w.y = w.y * 5.0
    w.cell_size = 1.0
    return w


CASES = {"sod16": ci.config0, "wall": wall_block, "behind": behind_block,
         "moving": moving_cloud, "slab": slab_cloud}


def horizon_pairs(w, R, t):
    """Oracle: {(i, j, mirror)} with |r_i - r_j| < R (j != i), and, with a wall at
    x_w(t), |r_i - (2 x_w - x_j, y_j, z_j)| < R; FP64 ((dx^2 + dy^2) + dz^2) < R^2."""
    cfg = O.make_cfg(w.eos, h=R / w.kappa, kappa=w.kappa)
    off, idx = O.neighbors(cfg, np.asarray(w.x), np.asarray(w.y), np.asarray(w.z))
    out = set()
    for i in range(w.n):
        for j in idx[off[i]:off[i + 1]]:
            out.add((i, int(j), False))
    if w.wall is not None:
        xw = w.wall[0] + w.wall[1] * t
        gx = 2.0 * xw - w.x
        for i in range(w.n):
            dx = gx - w.x[i]
            dy = w.y - w.y[i]
            dz = w.z - w.z[i]
            r2 = ((dx * dx) + (dy * dy)) + (dz * dz)
            for j in np.nonzero(r2 < R * R)[0]:
                out.add((i, int(j), True))
    return out


@pytest.mark.parametrize("case", ["sod16", "wall", "behind", "slab"])
def test_lists_are_the_horizon_pairs(case):
    w = CASES[case]()
    beta = 0.3
    print(f"[case] vlist build {case} n={w.n}", flush=True)
    params = P.Params.from_workload(w, reorder=True)
    g = P.state_from_workload(w, params, DEV, with_id=True)
    sc = P.StepScalars(DEV, t0=0.375)
    other = g.like()
    cap = 512  # behind the wall a particle has real and mirror partners all round
    count = torch.zeros(w.n, dtype=torch.int32, device=DEV)
    idx = torch.empty(w.n * cap, dtype=torch.int32, device=DEV)
    xref = torch.empty(3 * w.n, dtype=torch.float64, device=DEV)
    assert P.csph_vlist_build(g, other, params, sc, beta, cap, count, idx, xref) == 0
    torch.cuda.synchronize()
    ids = to_np(other.id)
    cnt = to_np(count)
    # 8-entry chunks: entry k of particle s at [k // 8, s, k % 8]
    lst = to_np(idx).reshape(cap // 8, w.n, 8).transpose(1, 0, 2).reshape(w.n, cap)
    got = set()
    for s in range(w.n):
        for e in lst[s, :cnt[s]]:
            j = int(e) & 0x7FFFFFFF
            got.add((int(ids[s]), int(ids[j]), bool(e < 0)))
    assert got == horizon_pairs(w, (1.0 + beta) * (w.kappa * w.h), 0.375)
    # reference positions are the renumbered positions
    xr = to_np(xref).reshape(3, w.n)
    assert np.array_equal(xr[0], w.x[ids]) and np.array_equal(xr[2], w.z[ids])


def test_list_overflow_reports_the_longest():
    w = ci.config0()
    params = P.Params.from_workload(w)
    g = P.state_from_workload(w, params, DEV)
    sc = P.StepScalars(DEV)
    count = torch.zeros(w.n, dtype=torch.int32, device=DEV)
    idx = torch.empty(w.n * 8, dtype=torch.int32, device=DEV)
    xref = torch.empty(3 * w.n, dtype=torch.float64, device=DEV)
    longest = P.csph_vlist_build(g, g.like(), params, sc, 0.3, 8, count, idx, xref)
    assert longest == int(to_np(count).max()) > 8


def _run(w, precision, beta, n_upd, steps, cap=None):
    params = P.Params.from_workload(w, precision=precision, reorder=True)
    g = P.state_from_workload(w, params, DEV, with_id=True)
    sc = P.StepScalars(DEV, t0=0.0)
    run = P.VerletRun(g, params, beta=beta, n_upd=n_upd, cap=cap)
    cfg = O.cfg_for(w, search=1)
    s = O.state_from(w, cfg)
    s0 = {k: v.copy() for k, v in s.items()}
    t = 0.0
    cnt = torch.empty(w.n, dtype=torch.int32, device=DEV)
    worst = 0.0
    for k in range(steps):
        st = run.step(sc, nbr_count=cnt)
        torch.cuda.synchronize()
        s, t, dt, ncount = O.step(cfg, s, t=t)
        got = st.numpy()
        ids = got["id"]
        assert np.array_equal(to_np(cnt).astype(np.int64), ncount[ids]), k
        # FP32 pair arithmetic gives the signal speed, hence dt, to FP32 accuracy
        dtol = 1e-13 if precision == "fp64" else 2e-6
        assert abs(to_np(sc.dt)[0] - dt) <= dtol * dt, (k, to_np(sc.dt)[0], dt)
        for f in ("x", "y", "z", "vx", "vy", "vz", "rho", "E"):
            a, b = got[f], s[f][ids]
            den = max(np.abs(b - s0[f][ids]).max(), 1e-300)
            worst = max(worst, float(np.abs(a - b).max() / den))
    return run, worst


@pytest.mark.parametrize("case", ["sod16", "wall", "behind", "moving", "slab"])
def test_verlet_run_fp64_follows_oracle(case):
    w = CASES[case]()
    print(f"[case] verlet fp64 {case} n={w.n}", flush=True)
    run, worst = _run(w, "fp64", beta=0.3, n_upd=5, steps=12)
    print("builds", run.builds, "worst rel", worst)
    assert worst <= 1e-10
    assert run.builds >= 3
    if case == "moving":
        assert run.builds > 3  # the displacement bound forced early rebuilds


@pytest.mark.parametrize("case", ["wall", "moving"])
def test_verlet_run_mixed_follows_oracle(case):
    w = CASES[case]()
    print(f"[case] verlet mixed {case} n={w.n}", flush=True)
    run, worst = _run(w, "mixed", beta=0.3, n_upd=5, steps=8)
    print("builds", run.builds, "worst rel", worst)
    assert worst <= 1e-4


@pytest.mark.parametrize("case", ["moving", "wall"])
def test_verlet_advance_batches_equal_single_steps(case):
    """advance(k) issues the list steps without waiting and lets the device guard stop a
    stale list; it gives bit for bit the states of k single steps (the same rebuilds at the
    same steps), and the control block's pair counts add up to the steps' neighbour counts."""
    w = CASES[case]()
    print(f"[case] verlet advance {case} n={w.n}", flush=True)
    params = P.Params.from_workload(w, precision="fp64", reorder=True)
    out = []
    for batched in (False, True):
        g = P.state_from_workload(w, params, DEV, with_id=True)
        sc = P.StepScalars(DEV, t0=0.0)
        run = P.VerletRun(g, params, beta=0.3, n_upd=5)
        cnt = torch.empty(w.n, dtype=torch.int32, device=DEV)
        total = 0
        if batched:
            st = run.advance(sc, 12, nbr_count=cnt)
        else:
            for _ in range(12):
                st = run.step(sc, nbr_count=cnt)
                total += int(cnt.sum().item())
        torch.cuda.synchronize()
        r = st.numpy()
        r.update(t=to_np(sc.t), tot=to_np(sc.totals))
        out.append((r, run.builds, run.pairs, total))
    (a, ba, pa, ta), (b, bb, pb, _) = out
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    assert ba == bb and pa == pb == ta
    if case == "moving":
        assert ba > 3  # the guard stopped lists before n_upd steps


def test_verlet_run_grows_a_small_cap():
    w = ci.config0()
    run, worst = _run(w, "fp64", beta=0.5, n_upd=4, steps=5, cap=8)
    assert run.cap > 8 and worst <= 1e-10
