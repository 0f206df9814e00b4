#!/usr/bin/env python3
"""Throughput of the contact-SPH hot path on one MI355X.

A step is one pass of the whole hot path over the particle set: mesh
bounds, cell binning and cell-ordered renumbering, pack + EOS, pair rates
(Riemann-solver contact flux), state update with the CFL time step and
compensated totals, and the Voronoi ownership of the new positions with
per-site particle and pair counts for 64 generators (computed by the update
kernel: csph_step_voronoi).

Default workload: porous-sample shock, 256^3 jittered lattice with seeded
spherical voids (radius 5, 30 % porosity, 11 743 903 particles), ideal gas
1.4, piston at x = 0 moving at +2, FP32 pair arithmetic with FP64 positions,
integration and totals.  The plain-FP64 GPU step is timed beside it.

Prints ONE JSON line.  `value` = directed pair interactions per second
(sum_i |N(i)| per step x steps per second) with the state resident in HBM,
over the workload's 100 steps from its initial state (the warm-up runs the
same loop on a throwaway copy).
"""
import argparse
import contextlib
import gc
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CSPH pair-interactions/s and steps/s at 16M particles; adjoint/forward time ratio"
OTHER_STEPS = 10  # steps of the pass that times the kernel groups other than the pair rates
PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector (published; FMA = 2, packed FP32 = 2x)
PEAK_HBM_GBS = 8000.0
# Algorithmic VALU work of the pair-flux step: 7 lane operations per candidate of the method's
# cell-list search over the 27 cells of size H around a particle (sec. 4.2; the neighbour
# test r^2 < H^2) and ~50 per interacting directed pair (Riemann solver, kernel slope, sums),
# against the chip's unpacked lane rate, 256 CUs x 64 lanes x 2.4 GHz = 39.3 T lane-ops/s.
OPS_PER_CANDIDATE = 7
OPS_PER_PAIR = 50
PEAK_LANE_TOPS = 256 * 64 * 2.4e9 / 1e12
# algorithmic FP32 operations per directed interacting pair: r, 1/r, e (3),
# q, 1-q, W' (4), v_L, v_R (10), S, 1/S, v* (6), P* (8), weight (1), the
# three sums (3 + 7 + 2) and the signal speed (3)
FLOP_PER_PAIR = 53


def cell27_candidates(x, y, z, H):
    """sum_i of the particles in the 3^3 mesh cells of size H around i's cell (i included):
    the candidates of the plain cell-list search with cells of the support's size."""
    import numpy as np
    c = [np.floor((a - a.min()) / H).astype(np.int64) for a in (x, y, z)]
    dims = [int(ci.max()) + 1 for ci in c]
    cnt = np.bincount((c[2] * dims[1] + c[1]) * dims[0] + c[0],
                      minlength=dims[0] * dims[1] * dims[2]).reshape(dims[2], dims[1], dims[0])
    pad = np.pad(cnt.astype(np.int64), 1)
    near = sum(pad[1 + a:1 + a + dims[2], 1 + b:1 + b + dims[1], 1 + c_:1 + c_ + dims[0]]
               for a in (-1, 0, 1) for b in (-1, 0, 1) for c_ in (-1, 0, 1))
    return int((cnt.astype(np.int64) * near).sum())


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="porous", choices=["porous", "voidfree"])
    ap.add_argument("--fp64-steps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slab", type=float, default=96.0,
                    help="oracle sample: particles with x < this (same workload)")
    ap.add_argument("--no-extra", dest="extra", action="store_false",
                    help="skip the void-free twin and the plate-impact runs")
    ap.add_argument("--verlet-steps", type=int, default=10,
                    help="also time this many Verlet-list steps (0: skip)")
    ap.add_argument("--no-adjoint", dest="adjoint", action="store_false",
                    help="skip the adjoint/forward ratio of the 64^3 checkpointed rollout")
    ap.add_argument("--cell", type=float, default=1.0,
                    help="mesh cell size in lattice spacings (results do not depend on it)")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="first copy a buffer of this many GiB three times (counter calibration)")
    ap.add_argument("--no-collision", dest="collision", action="store_false",
                    help="skip the 64 M-particle collision leg")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


@contextlib.contextmanager
def collector_off():
    """Python's cyclic garbage collector off, after a full collection, for a timed region
    including its closing device synchronisation: a collection pause (tens of ms with torch
    loaded) must not land between the start and the stop of the clock."""
    gc.collect()
    gc.disable()
    try:
        yield
    finally:
        gc.enable()


class Runner:
    """Step loop with every buffer allocated up front (nothing is allocated while timed)."""

    def __init__(self, P, torch, state, params, sites, ws, sc):
        n = state.n
        self.P, self.params, self.sites, self.ws, self.sc = P, params, sites, ws, sc
        self.cnt = torch.empty(n, dtype=torch.int32, device="cuda")
        self.owner = torch.empty(n, dtype=torch.int32, device="cuda")
        self.site_particles = torch.empty(sites.shape[0], dtype=torch.int64, device="cuda")
        self.site_pairs = torch.empty(sites.shape[0], dtype=torch.int64, device="cuda")
        self.pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
        self.state, self.other = state, state.like()

    def run(self, k, count_pairs=True):
        """k steps of (csph_step, voronoi_assign); directed pairs summed on the device."""
        P = self.P
        for _ in range(k):
            # the step and the Voronoi ownership of its result in one call (the ownership is
            # computed by the step's update kernel; bit-identical to voronoi_assign after it)
            out = P.csph_step_voronoi(self.state, self.params, self.sc, self.sites, self.owner,
                                      self.site_particles, self.site_pairs, s_out=self.other,
                                      nbr_count=self.cnt, ws=self.ws)
            if count_pairs:
                self.pairs += self.site_pairs.sum()
            self.state, self.other = out, self.state


def balance_timing(P, torch, run, sites, iters=10):
    """Balancer iteration (subdomain statistics + generator move) on the final state of the
    timed run with its 64 generators: HIP-event time per iteration."""
    bp = P.BalanceParams(sigma=0.5, theta=0.25, gamma=1.0, dsh=3.0, load="pairs")
    s = run.state
    g = sites.clone()
    st = P.csph_balance_stats(s["x"], s["y"], s["z"], run.owner, g, bp.dsh, nbr_count=run.cnt)
    P.csph_balance_move(g, st, bp)
    torch.cuda.synchronize()
    P.profile_enable(True)
    P.profile_read()
    for _ in range(iters):
        st = P.csph_balance_stats(s["x"], s["y"], s["z"], run.owner, g, bp.dsh, nbr_count=run.cnt)
        P.csph_balance_move(g, st, bp)
    torch.cuda.synchronize()
    launches, ms = P.profile_read()["balance"]
    P.profile_enable(False)
    adj = P.adjacency_matrix(st["adjacency"], g.shape[0])
    return {"ms_per_iteration": ms / iters, "sites": int(g.shape[0]), "iterations": iters,
            "touching_pairs": int(adj.sum().item()) // 2,
            "note": "stats pass over all particles + one-workgroup generator move"}


def impact_run(P, torch, ci, steps):
    """Plate impact (589 824 particles, no walls: a closed system), ``steps`` steps from the
    initial state in each precision, and in mixed precision with the target's lateral faces
    periodic (the paper's plate tests are periodic across the impact direction): time per
    step, pair interactions/s, and the drift of the compensated totals of momentum and energy
    from the first step's state to the last."""
    w = ci.config1()
    out = {"workload": w.name, "particles": w.n, "steps": steps}
    for prec in ("mixed", "fp64", "mixed_periodic_xy"):
        over = {}
        if prec == "mixed_periodic_xy":
            over = dict(periodic=3, box=((0.0, 0.0, 0.0), (128.0, 128.0, 0.0)))
        params = P.Params.from_workload(w, precision=prec[:5], reorder=True, cell_size=1.0,
                                        **over)
        cnt = torch.empty(w.n, dtype=torch.int32, device="cuda")
        pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
        # warm-up on a throwaway copy (it also sizes the workspace, so nothing is allocated
        # while timed), then the timed run from the initial state
        ws = P.Workspace("cuda")
        for warm in (True, False):
            state = P.state_from_workload(w, params, "cuda", with_id=False)
            other = state.like()
            sc = P.StepScalars("cuda")
            k = 3 if warm else steps
            pairs.zero_()
            with collector_off():
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for i in range(k):
                    o = P.csph_step(state, params, sc, s_out=other, nbr_count=cnt, ws=ws)
                    pairs += cnt.sum()  # the warm-up runs the timed loop's own operations
                    if i == 0 and not warm:
                        tot_first = sc.totals.clone()
                    state, other = o, state
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
        t1 = sc.totals.cpu().numpy()
        t0_ = tot_first.cpu().numpy()
        tot = lambda t, a: float(t[2 * a]) + float(t[2 * a + 1])
        mom_scale = float((state["m"] * (state["vx"].abs() + state["vy"].abs() +
                                         state["vz"].abs())).sum())
        dmom = max(abs(tot(t1, a) - tot(t0_, a)) for a in (1, 2, 3)) / mom_scale
        de = (tot(t1, 4) - tot(t0_, 4)) / abs(tot(t0_, 4))
        out[prec] = {"ms_per_step": 1e3 * el / steps, "pairs_per_s": int(pairs.item()) / el,
                     "momentum_drift_rel": dmom, "energy_drift_rel": de,
                     "t_end": float(sc.t.item())}
        del state, other, ws
        torch.cuda.empty_cache()
    out["mixed_graph"] = impact_graph_run(P, torch, w, steps)
    out["mixed_speedup_over_fp64"] = out["fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"]
    out["note"] = ("drifts of the compensated totals sum(m v), sum(m E) between the states after "
                   "step 1 and the last step, relative to sum(m|v|) and |sum(m E)|")
    return out


def impact_graph_run(P, torch, w, steps, k=10):
    """The plate impact with periodic lateral faces (the bounded domain a fixed mesh suits),
    mixed precision, on a fixed mesh (csph_step_mesh: no bounds pass, no host synchronisation)
    covering the periodic box laterally and z from -96 to 96: ``k`` steps captured in one graph
    and replayed steps / k times from the initial state.  Time per step, and the particles that
    left the mesh (0: every step was exact; compare with the eager periodic leg)."""
    box = ((0.0, 0.0, -96.0), (128.0, 128.0, 96.0))
    params = P.Params.from_workload(w, precision="mixed", reorder=True, cell_size=1.0,
                                    periodic=3, box=box)
    mesh = P.domain_mesh(box[0], box[1], params)
    ws = P.Workspace("cuda")
    warm = P.state_from_workload(w, params, "cuda", with_id=False)
    P.csph_step_mesh(warm, params, P.StepScalars("cuda"), mesh, s_out=warm.like(), ws=ws)
    del warm
    a = P.state_from_workload(w, params, "cuda", with_id=False)
    b = a.like()
    sc = P.StepScalars("cuda")
    outside = torch.zeros(1, dtype=torch.int64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        for i in range(k):
            src, dst = (a, b) if i % 2 == 0 else (b, a)
            P.csph_step_mesh(src, params, sc, mesh, s_out=dst, outside=outside, ws=ws)
    with collector_off():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps // k):
            graph.replay()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    out = {"ms_per_step": 1e3 * el / (steps // k * k), "steps_per_graph": k,
           "mesh": {"origin": list(mesh.origin), "dims": list(mesh.dims), "cell": mesh.cell},
           "outside_after_run": int(outside.item()), "t_end": float(sc.t.item())}
    del graph, a, b, ws
    torch.cuda.empty_cache()
    return out


def rk2_run(P, torch, w, cell, steps):
    """The two-stage Runge-Kutta step (two rate evaluations per step) on the porous shock in
    mixed precision, ``steps`` steps from the initial state after 3 warm-up steps on a
    throwaway copy: time per step and the directed pairs of the first evaluation."""
    params = P.Params.from_workload(w, precision="mixed", reorder=True, cell_size=cell,
                                    integrator="rk2")
    cnt = torch.empty(w.n, dtype=torch.int32, device="cuda")
    pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = P.Workspace("cuda")
    for warm in (True, False):
        state = P.state_from_workload(w, params, "cuda", with_id=False)
        other = state.like()
        sc = P.StepScalars("cuda")
        k = 3 if warm else steps
        P.profile_enable(True)
        P.profile_read()
        with collector_off():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(k):
                o = P.csph_step(state, params, sc, s_out=other, nbr_count=cnt, ws=ws)
                if not warm:
                    pairs += cnt.sum()
                state, other = o, state
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        prof = P.profile_read()
        P.profile_enable(False)
    behind = int((state["x"] < w.wall[0] + w.wall[1] * float(sc.t.item())).sum().item())
    out = {"workload": w.name, "particles": w.n, "steps": steps, "precision": "mixed",
           "rate_evaluations_per_step": 2, "ms_per_step": 1e3 * el / steps,
           "pairs_per_step": int(pairs.item()) / steps,
           "pairs_per_s": 2 * int(pairs.item()) / el,
           "kernel_ms": {g: round(v[1] / max(v[0], 1), 4) for g, v in prof.items() if v[0] > 0},
           "t_end": float(sc.t.item()), "behind_wall_after_run": behind,
           "note": "pairs_per_s counts both evaluations (the second's pairs taken equal to the "
                   "first's); kernel_ms are per launch, two launches of bin, pack and rates "
                   "per step"}
    del state, other, ws
    torch.cuda.empty_cache()
    return out


def paper_mode_run(P, torch, ci, steps, nx=256, ny=256, nz=48):
    """The paper's material mode at scale: an aluminium plate (v_z = -0.5 km/s) on a lead
    plate, Mie-Grueneisen (sec. 5 parameters, g/cc, km/s, GPa), support kappa (d_i + d_j)/2
    with kappa = 1.936 and d = (m/rho)^(1/3); ``steps`` steps from the initial state in each
    precision after 3 warm-up steps on a throwaway copy."""
    import numpy as np
    w = ci.mg_plates(nx, ny, nz)
    d = np.cbrt(w.m / w.rho)
    out = {"workload": w.name, "particles": w.n, "steps": steps,
           "kappa": 1.936, "cell": 1.0}
    for prec in ("mixed", "fp64"):
        params = P.Params.from_workload(w, precision=prec, reorder=True, h_mode="pair",
                                        kappa=1.936, cell_size=1.0, wall=None)
        cnt = torch.empty(w.n, dtype=torch.int32, device="cuda")
        pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
        ws = P.Workspace("cuda")  # sized by the warm-up, so nothing is allocated while timed
        for warm in (True, False):
            state = P.state_from_workload(w, params, "cuda", with_id=False)
            state.d = torch.as_tensor(d, dtype=torch.float64, device="cuda")
            other = state.like()
            sc = P.StepScalars("cuda")
            k = 3 if warm else steps
            pairs.zero_()
            with collector_off():
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for i in range(k):
                    o = P.csph_step(state, params, sc, s_out=other, nbr_count=cnt, ws=ws)
                    pairs += cnt.sum()  # the warm-up runs the timed loop's own operations
                    state, other = o, state
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
        out[prec] = {"ms_per_step": 1e3 * el / steps, "pairs_per_s": int(pairs.item()) / el,
                     "pairs_per_step": int(pairs.item()) / steps, "t_end": float(sc.t.item())}
        del state, other, ws
        torch.cuda.empty_cache()
    out["mixed_speedup_over_fp64"] = out["fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"]
    return out


def voidfree_run(P, torch, ci, steps, cell):
    """The void-free 256^3 twin (16 777 216 particles), mixed, whole step with Voronoi: its
    ``steps`` steps from the initial state, after 3 warm-up steps on a throwaway copy."""
    w = ci.config2(voids=False)
    params = P.Params.from_workload(w, precision="mixed", reorder=True, cell_size=cell)
    sites = torch.as_tensor(w.sites, dtype=torch.float64, device="cuda")
    ws = P.Workspace("cuda")
    warm = Runner(P, torch, P.state_from_workload(w, params, "cuda", with_id=False), params,
                  sites, ws, P.StepScalars("cuda"))
    with collector_off():
        warm.run(3)
        torch.cuda.synchronize()
    del warm
    state = P.state_from_workload(w, params, "cuda", with_id=False)
    sc = P.StepScalars("cuda")
    run = Runner(P, torch, state, params, sites, ws, sc)
    torch.cuda.synchronize()
    run.pairs.zero_()
    with collector_off():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run.run(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    npairs = int(run.pairs.item())
    out = {"workload": w.name, "particles": w.n, "steps": steps, "ms_per_step": 1e3 * el / steps,
           "steps_per_s": steps / el, "pairs_per_s": npairs / el}
    del run, state
    torch.cuda.empty_cache()
    return out


def verlet_timing(P, torch, w, cell, steps, beta=0.3, n_upd=10):
    """Verlet-list steps (lists within (1 + beta) H, rebuilt every n_upd steps or when the
    displacement bound requires) on the same workload, mixed precision: the rebuilds are
    inside the timed steps."""
    params = P.Params.from_workload(w, precision="mixed", reorder=True, cell_size=cell)
    state = P.state_from_workload(w, params, "cuda", with_id=False)
    sc = P.StepScalars("cuda")
    run = P.VerletRun(state, params, beta=beta, n_upd=n_upd)
    run.advance(sc, 2)
    torch.cuda.synchronize()
    b0, p0 = run.builds, run.pairs
    P.profile_enable(True)
    P.profile_read()
    with collector_off():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # list steps issued without waiting; one synchronisation per batch (the control
        # block's read), the device guard deciding the rebuilds
        run.advance(sc, steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    prof = P.profile_read()
    P.profile_enable(False)
    npairs = run.pairs - p0
    out = {"metric_value": npairs / el, "unit": "pair-interactions/s", "ms_per_step": 1e3 * el / steps,
           "steps": steps, "beta": beta, "n_upd": n_upd, "rebuilds": run.builds - b0,
           "list_cap": run.cap,
           "kernel_ms": {g: round(v[1] / max(v[0], 1), 4) for g, v in prof.items() if v[0] > 0},
           "note": "rebuild (bin + renumber + list build) counted in 'neighbors' and 'bin'"}
    del run, state
    torch.cuda.empty_cache()
    return out


def verlet_vs_search(P, torch, w, steps, beta=0.3, n_upd=10):
    """Verlet-list steps against the per-step search on one workload (mixed precision, both
    from the initial state after 3 warm-up steps on a throwaway copy): a list step needs no
    mesh, no binning and no host synchronisation, so it pays where particles move little per
    step and launches and the mesh synchronisation weigh on the per-step search."""
    params = P.Params.from_workload(w, precision="mixed", reorder=True)
    out = {"workload": w.name, "particles": w.n, "steps": steps, "beta": beta, "n_upd": n_upd,
           "cfl": w.cfl}
    ws = P.Workspace("cuda")
    for warm in (True, False):
        state = P.state_from_workload(w, params, "cuda", with_id=True)
        other = state.like()
        sc = P.StepScalars("cuda")
        cnt = torch.empty(w.n, dtype=torch.int32, device="cuda")
        k = 3 if warm else steps
        with collector_off():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(k):
                o = P.csph_step(state, params, sc, s_out=other, nbr_count=cnt, ws=ws)
                state, other = o, state
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
    out["search_ms_per_step"] = 1e3 * el / steps
    x_search = state["x"][torch.argsort(state.id)].clone()
    del state, other
    for warm in (True, False):
        state = P.state_from_workload(w, params, "cuda", with_id=True)
        sc = P.StepScalars("cuda")
        run = P.VerletRun(state, params, beta=beta, n_upd=n_upd, ws=ws)
        k = 3 if warm else steps
        with collector_off():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run.advance(sc, k)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
    out["verlet_ms_per_step"] = 1e3 * el / steps
    out["rebuilds"] = run.builds
    out["verlet_over_search"] = out["verlet_ms_per_step"] / out["search_ms_per_step"]
    # the same steps through both paths (mixed precision: the two walks round their FP32
    # offsets differently, so the positions agree to the FP32 rate tolerance, not bitwise)
    st = run.state
    out["max_abs_x_difference"] = float((st["x"][torch.argsort(st.id)] - x_search).abs().max())
    del run, state, ws
    torch.cuda.empty_cache()
    return out


def collision_run(P, torch, ci, steps=50, window=5):
    """Heterogeneous collision (64 000 000 particles): ``steps`` mixed steps from the initial
    state (after 3 warm-up steps on a throwaway copy), and the adjoint of the last ``window``
    steps w.r.t. the velocities at their start (the FP64 window recomputed from one checkpoint;
    objective: z-momentum of the dense body), as adjoint/forward wall-time ratio."""
    t0 = time.perf_counter()
    w = ci.config4()
    log(f"collision: {w.n} particles ({time.perf_counter() - t0:.1f} s to generate)")
    params = P.Params.from_workload(w, precision="mixed", reorder=True, cell_size=1.0)
    fp64_window = P.Params.from_workload(w, precision="fp64", cell_size=1.0)
    gamma = torch.tensor([e[1] for e in w.eos], dtype=torch.float64, device="cuda")
    ws = P.Workspace("cuda")
    cnt = torch.empty(w.n, dtype=torch.int32, device="cuda")
    pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    warm = P.state_from_workload(w, params, "cuda", with_id=False)
    other = warm.like()
    sc = P.StepScalars("cuda")
    for i in range(3):
        warm, other = P.csph_step(warm, params, sc, s_out=other, nbr_count=cnt, ws=ws), warm
    torch.cuda.synchronize()
    state = P.state_from_workload(w, params, "cuda", with_id=False)
    n = w.n
    del w, warm
    sc = P.StepScalars("cuda")
    ckpt = None
    el = 0.0
    with collector_off():
        for seg in (steps - window, window):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(seg):
                state, other = P.csph_step(state, params, sc, s_out=other, nbr_count=cnt,
                                           ws=ws), state
                pairs += cnt.sum()
            torch.cuda.synchronize()
            el += time.perf_counter() - t1
            if ckpt is None:  # the window's start (outside the timed region)
                ckpt = {k: state.t[k].clone() for k in ("x", "y", "z", "vx", "vy", "vz", "rho",
                                                         "E", "m")}
                ckpt["mat"] = state.mat.clone()
    out = {"workload": f"collision_{n}", "particles": n, "steps": steps,
           "ms_per_step": 1e3 * el / steps, "steps_per_s": steps / el,
           "pairs_per_s": int(pairs.item()) / el, "pairs_per_step": int(pairs.item()) / steps,
           "nonphys": int(sc.nonphys.item())}
    del state, other, ws
    torch.cuda.empty_cache()
    base = {k: ckpt[k] for k in ("x", "y", "z", "rho", "E", "m", "mat")}
    v0 = [ckpt[k].requires_grad_(True) for k in ("vx", "vy", "vz")]
    body_a = base["mat"] == 1
    info = {}
    with collector_off():
        res = P.rollout(*v0, gamma, base, fp64_window, window, window, info=info)
        J = (res["vz"][body_a] * base["m"][body_a]).sum()
        torch.autograd.grad(J, v0)
        torch.cuda.synchronize()
    out["adjoint_window"] = {"steps": window, "precision": "fp64", "checkpoints": 1,
                             "forward_s": round(info["forward_s"], 5),
                             "backward_s": round(info["backward_s"], 5),
                             "ratio": info["backward_s"] / info["forward_s"]}
    del res, J, v0, base, ckpt
    torch.cuda.empty_cache()
    return out


# Algorithmic HBM bytes per particle of the memory-bound kernel groups of a step (what the
# method must move through memory, not what an implementation happens to move):
#   bin:       positions read once (24), the cell order written (4) and the cell ranges
#              (4 per cell, added per particle from the mesh size);
#   pack:      the state gathered (72 + mat 4 + id 8 + perm 4) and written in cell order
#              (72 + 4 + 8) with the 48-byte FP32 pair record;
#   integrate: state (72) and rates (40) read, the 64 evolving bytes written, and with the
#              Voronoi ownership of the new positions (one kernel) the pair count (4) read and
#              the owner (4) written;
#   voronoi:   positions (24) and the pair count (4) read, the owner (4) written.
HBM_BYTES = {"bin": 28, "pack": 88 + 132, "integrate": 112 + 64 + 8, "voronoi": 32}


def hbm_block(kernel_ms, n, ncell):
    out = {}
    for g, b in HBM_BYTES.items():
        if g not in kernel_ms or kernel_ms[g] <= 0:
            continue
        per = b + (4.0 * ncell / n if g == "bin" else 0.0)
        gbs = per * n / (kernel_ms[g] * 1e-3) / 1e9
        out[g] = {"ms": kernel_ms[g], "alg_bytes_per_particle": round(per, 2),
                  "achieved_GBps": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4)}
    return out


KERNEL_SOURCES = ("k_rates.hip", "stencil.h", "csph_internal.h")


def kernel_source_sha(texts=None):
    """sha256 of the rate kernel's sources with // comments and blank lines removed (comment
    edits do not change the kernel the counters were taken on)."""
    import hashlib
    if texts is None:
        csrc = os.path.join(ROOT, "paper_1805_05128_amd", "csrc")
        texts = [open(os.path.join(csrc, f), "rb").read().decode() for f in KERNEL_SOURCES]
    code = []
    for t in texts:
        for line in t.split("\n"):
            line = re.sub(r"//.*$", "", line).rstrip()
            if line:
                code.append(line)
    return hashlib.sha256("\n".join(code).encode()).hexdigest()


def traffic_from_profile():
    """HBM bytes per launch of the pair-rate kernel from the committed counter summary,
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_rates32_porous256.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    fields = dict(re.findall(r"^- (\w+): (\S+)$", text, re.M))
    sha = kernel_source_sha()
    if fields.get("source_sha256") != sha:
        return None
    return {"read_bytes": float(fields["read_bytes_per_launch"]),
            "write_bytes": float(fields["write_bytes_per_launch"]),
            "bytes": float(fields["read_bytes_per_launch"]) + float(fields["write_bytes_per_launch"])}


def adjoint_ratio(P, torch, ci):
    """Adjoint/forward wall-time ratio of the checkpointed 64^3 Sod rollout
    (100 FP64 steps, checkpoint every 10, objective: x-momentum beyond x = 48)."""
    import numpy as np
    w = ci.config3()
    params = P.Params.from_workload(w)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64), device="cuda").contiguous()
    base = dict(x=t(w.x), y=t(w.y), z=t(w.z), rho=t(w.rho), p=t(w.p), m=t(w.m),
                mat=torch.as_tensor(w.mat, dtype=torch.int32, device="cuda"))
    gamma = torch.tensor([w.eos[0][1]], dtype=torch.float64, device="cuda", requires_grad=True)
    best = None
    for _ in range(2):  # the first rollout also warms the library's code paths
        v0 = [t(a).requires_grad_(True) for a in (w.vx, w.vy, w.vz)]
        info = {}
        with collector_off():
            out = P.rollout(*v0, gamma, base, params, w.steps, 10, info=info)
            mask = out["x"].detach() > 48.0
            J = (out["vx"][mask] * base["m"][mask]).sum()
            torch.autograd.grad(J, v0 + [gamma])
        r = {"ratio": info["backward_s"] / info["forward_s"], "forward_s": info["forward_s"],
             "backward_s": info["backward_s"]}
        best = r
    # the same rollout differentiated with its CFL steps (csph_step_vjp_cfl: one more FP64
    # rate evaluation and one host synchronisation per step)
    for _ in range(2):
        v0 = [t(a).requires_grad_(True) for a in (w.vx, w.vy, w.vz)]
        info = {}
        with collector_off():
            out = P.rollout(*v0, gamma, base, params, w.steps, 10, info=info, cfl_adjoint=True)
            mask = out["x"].detach() > 48.0
            J = (out["vx"][mask] * base["m"][mask]).sum()
            torch.autograd.grad(J, v0 + [gamma])
        best["ratio_cfl_adjoint"] = info["backward_s"] / info["forward_s"]
    return {"workload": w.name, "particles": w.n, "steps": w.steps, "checkpoint_every": 10,
            "precision": "fp64", **{k: round(v, 5) for k, v in best.items()}}


def cpu_baseline(w, slab):
    import numpy as np

    import oracle as O
    keep = w.x < slab
    sub = type(w)(**{**w.__dict__})
    for k in ("x", "y", "z", "vx", "vy", "vz", "rho", "p", "m", "mat"):
        setattr(sub, k, np.ascontiguousarray(getattr(w, k)[keep]))
    cfg = O.cfg_for(sub, search=1)
    s = O.state_from(sub, cfg)
    t0 = time.perf_counter()
    _, _, _, cnt = O.step(cfg, s, 0.0)
    el = time.perf_counter() - t0
    pairs = int(cnt.sum())
    return {"value": pairs / el, "unit": "pair-interactions/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"one full oracle step (cell-list search, FP64) on the slab x < {slab:g} of "
                      f"the same porous workload: {sub.n} particles, {pairs} directed pairs, "
                      f"{el:.2f} s",
            "steps_per_s_sample": 1.0 / el}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "decomposition (one Voronoi subdomain per GPU) is designed, not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import csph_inputs as ci
    import paper_1805_05128_amd as P

    if args.copy_probe > 0:
        nbytes = int(args.copy_probe * (1 << 30))
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: 3 copies of {nbytes} bytes")
        del src, dst
    t_gen = time.perf_counter()
    w = ci.config2(voids=(args.workload == "porous"))
    log(f"workload {w.name}: {w.n} particles ({time.perf_counter() - t_gen:.1f} s to generate)")
    torch.cuda.set_device(0)
    sites = torch.as_tensor(w.sites, dtype=torch.float64, device="cuda")
    ws = P.Workspace("cuda")

    results = {}
    for prec, k in (("mixed", args.steps), ("fp64", args.fp64_steps)):
        if k <= 0:
            continue
        params = P.Params.from_workload(w, precision=prec, reorder=True, cell_size=args.cell)
        # warm-up: the same loop on a throwaway copy of the initial state (every kernel and
        # code path loaded, the event pool warmed); it also gives the totals after step 1
        P.profile_enable(True)
        tot0 = None
        if args.warmup > 0:
            wsc = P.StepScalars("cuda")
            wrun = Runner(P, torch, P.state_from_workload(w, params, "cuda", with_id=True),
                          params, sites, ws, wsc)
            with collector_off():
                wrun.run(1)
                tot0 = wsc.totals.clone()
                wrun.run(args.warmup - 1)
                torch.cuda.synchronize()
            tot0 = tot0.cpu().numpy()
            del wrun
        # the timed run: k steps of the workload from its initial state
        state = P.state_from_workload(w, params, "cuda", with_id=True)
        sc = P.StepScalars("cuda")
        run = Runner(P, torch, state, params, sites, ws, sc)
        torch.cuda.synchronize()
        # inside the timed steps only the pair-rate kernel records events (the roofline's
        # kernel); the other groups are timed in a pass of their own below
        P.profile_groups(["rates"])
        P.profile_read()
        run.pairs.zero_()
        with collector_off():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run.run(k)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        prof = P.profile_read()
        # the other kernel groups: OTHER_STEPS further steps from the timed run's final state
        # on a throwaway copy (in cell order, as the timed steps' inputs were), every group
        # timed (untimed as a whole)
        P.profile_groups(None)
        cp = run.state.like()
        for key, v in run.state.t.items():
            cp.t[key].copy_(v)
        for key in ("mat", "d", "id"):
            if getattr(cp, key) is not None:
                getattr(cp, key).copy_(getattr(run.state, key))
        orun = Runner(P, torch, cp, params, sites, ws,
                      P.StepScalars("cuda", t0=float(sc.t.item())))
        with collector_off():
            orun.run(OTHER_STEPS, count_pairs=False)
            torch.cuda.synchronize()
        other = P.profile_read()
        del orun
        prof = {g: (v if g == "rates" else other[g]) for g, v in prof.items()}
        P.profile_enable(False)
        tot1 = sc.totals.cpu().numpy()
        npairs = int(run.pairs.item())
        if prec == "mixed":
            results["balance"] = balance_timing(P, torch, run, sites)
            # the plain 27-cell search's candidates, mean of the first and the last state
            H = w.kappa * w.h
            st = run.state
            cand_end = cell27_candidates(*(st[a].cpu().numpy() for a in ("x", "y", "z")), H)
            results["candidates"] = 0.5 * (cell27_candidates(w.x, w.y, w.z, H) + cand_end)
            # cells of the step's mesh (unit cells on the final state's extent)
            ext = [float(st[a].max() - st[a].min()) for a in ("x", "y", "z")]
            results["ncell"] = int(np.prod([int(e / args.cell) + 2 for e in ext]))
        st = run.state
        t_end = float(sc.t.item())
        behind = int((st["x"] < w.wall[0] + w.wall[1] * t_end).sum().item())
        results[prec] = dict(ms=1e3 * el / k, pairs_per_step=npairs / k, el=el, k=k, prof=prof,
                             nonphys=int(sc.nonphys.item()), t=t_end,
                             tot0=tot0, tot1=tot1, behind=behind)
        log(f"{prec}: {1e3 * el / k:.3f} ms/step, {npairs / el:.3e} pairs/s, "
            f"rates kernel {prof['rates'][1] / max(prof['rates'][0], 1):.3f} ms")
        del state, run
        torch.cuda.empty_cache()

    m = results["mixed"]
    rates_launches, rates_ms = m["prof"]["rates"]
    rates_avg_s = rates_ms / max(rates_launches, 1) / 1e3
    cand = results["candidates"]
    lane_ops = OPS_PER_CANDIDATE * cand + OPS_PER_PAIR * m["pairs_per_step"]
    achieved = lane_ops / rates_avg_s / 1e12
    pair_tflops = FLOP_PER_PAIR * m["pairs_per_step"] / rates_avg_s / 1e12
    kernels = {g: round(v[1] / max(v[0], 1), 4) for g, v in m["prof"].items() if v[0] > 0}
    traffic = traffic_from_profile()
    # per particle the pair-rate kernel must read its 48 B FP32 record, FP64 position (24 B)
    # and density (8 B), and write five FP64 rates, the signal speed and the count (52 B)
    alg_bytes = w.n * (80 + 52)
    e0 = m["tot0"][8] + m["tot0"][9] if m["tot0"] is not None else 0.0
    e1 = m["tot1"][8] + m["tot1"][9]
    line = {
        "metric": METRIC,
        "value": m["pairs_per_step"] * 1e3 / m["ms"],
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms"],
        "steps_per_s": 1e3 / m["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair arithmetic, f64 positions/integration/totals",
        "data": "synthetic",
        "config": {"workload": w.name, "particles": w.n, "lattice": "256^3, 30% voids r=5",
                   "support": "2h = 3 spacings", "piston": "x=0, v=+2", "voronoi_sites": 64,
                   "eos": "ideal gas 1.4", "cfl": 0.3, "cell": args.cell},
        "pairs_per_step": m["pairs_per_step"],
        "kernel_ms": kernels,
        "kernel_ms_windows": {"rates": f"the {args.steps} timed steps",
                              "others": f"{OTHER_STEPS} further steps from the timed "
                                        "run's final state on a throwaway copy (their events "
                                        "kept out of the timed steps)"},
        "roofline": {"bound": "alu", "kernel": "k_rates32 (pair rates, FP32)",
                     "achieved": achieved, "peak": PEAK_LANE_TOPS, "unit": "T lane-op/s",
                     "frac": achieved / PEAK_LANE_TOPS,
                     "achieved_is": "algorithmic-equivalent work (the method's 27-cell search "
                                    "and pair arithmetic) / measured kernel time, not counted "
                                    "instructions: the kernel tests fewer candidates (chord-"
                                    "clipped rows) and issues more per pair",
                     "kernel_ms_window": rates_avg_s * 1e3,
                     "window": f"the {args.steps} timed steps (HIP events on the kernel's "
                               "stream)",
                     "hbm_view": {"alg_bytes": alg_bytes,
                                  "achieved_GBps": alg_bytes / rates_avg_s / 1e9,
                                  "frac": alg_bytes / rates_avg_s / 1e9 / PEAK_HBM_GBS},
                     "traffic": traffic["bytes"] if traffic else None,
                     "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE x2 + WRITE_SIZE)",
                     "algorithmic_bytes": alg_bytes,
                     "algorithmic_lane_ops": lane_ops,
                     "work": f"{OPS_PER_CANDIDATE} x {cand:.4g} candidates of the 27-cell search "
                             f"(cells of size H) + {OPS_PER_PAIR} x {m['pairs_per_step']:.4g} "
                             "directed pairs per launch",
                     "pair_flops": {"flop_per_pair": FLOP_PER_PAIR, "achieved": pair_tflops,
                                    "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                                    "frac": pair_tflops / PEAK_FP32_TFLOPS}},
        "energy_total_rel_change": (e1 - e0) / abs(e0) if e0 else None,
        "nonphys": m["nonphys"],
        "behind_wall_after_run": m["behind"],
        "hbm": {"peak_GBps": PEAK_HBM_GBS,
                "note": "memory-bound kernel groups of the mixed step: algorithmic bytes per "
                        "particle / HIP-event time; the step as a whole is bound by the "
                        "pair-rate kernel's instruction issue, so its HBM fraction is low",
                "kernels": hbm_block(kernels, w.n, results["ncell"])},
    }
    if "fp64" in results:
        f = results["fp64"]
        line["fp64"] = {"ms_per_step": f["ms"], "value": f["pairs_per_step"] * 1e3 / f["ms"],
                        "rates_kernel_ms": f["prof"]["rates"][1] / max(f["prof"]["rates"][0], 1),
                        "kernel_ms": {g: round(v[1] / max(v[0], 1), 4)
                                      for g, v in f["prof"].items() if v[0] > 0}}
        line["mixed_speedup_over_fp64"] = f["ms"] / m["ms"]
    line["unique_pairs_per_s"] = line["value"] / 2.0
    if "balance" in results:
        line["balance"] = results["balance"]
    if args.extra:
        log("void-free 256^3 twin ...")
        line["voidfree"] = voidfree_run(P, torch, ci, 100, args.cell)
        log(f"void-free: {line['voidfree']['ms_per_step']:.3f} ms/step")
        log("plate impact, both precisions ...")
        line["impact"] = impact_run(P, torch, ci, 200)
        log(f"impact mixed {line['impact']['mixed']['ms_per_step']:.3f} ms/step, "
            f"fp64 {line['impact']['fp64']['ms_per_step']:.3f} ms/step, mixed on a fixed mesh "
            f"in graphs {line['impact']['mixed_graph']['ms_per_step']:.3f} ms/step")
        log("Mie-Grueneisen plates, pair-averaged support, both precisions ...")
        line["paper_mode"] = paper_mode_run(P, torch, ci, 20)
        log(f"paper mode mixed {line['paper_mode']['mixed']['ms_per_step']:.3f} ms/step, "
            f"fp64 {line['paper_mode']['fp64']['ms_per_step']:.3f} ms/step")
        log("two-stage Runge-Kutta steps ...")
        line["rk2"] = rk2_run(P, torch, w, args.cell, 20)
        log(f"rk2 mixed {line['rk2']['ms_per_step']:.3f} ms/step")
    if args.extra and args.collision:
        log("two-body collision, 64 M particles ...")
        line["collision"] = collision_run(P, torch, ci)
        log(f"collision: {line['collision']['ms_per_step']:.3f} ms/step, adjoint/forward "
            f"{line['collision']['adjoint_window']['ratio']:.3f}")
    if args.verlet_steps > 0:
        log("Verlet-list steps ...")
        line["verlet"] = verlet_timing(P, torch, w, args.cell, args.verlet_steps)
        log(f"verlet: {line['verlet']['ms_per_step']:.3f} ms/step, "
            f"{line['verlet']['rebuilds']} rebuilds in {args.verlet_steps} steps")
        log("Verlet-list steps against the per-step search, Sod 64^3 ...")
        line["verlet_sod64"] = verlet_vs_search(P, torch, ci.config3(), 100)
        log(f"sod64: search {line['verlet_sod64']['search_ms_per_step']:.3f} ms/step, lists "
            f"{line['verlet_sod64']['verlet_ms_per_step']:.3f} ms/step, "
            f"{line['verlet_sod64']['rebuilds']} rebuilds")
    if args.adjoint:
        log("adjoint rollout ...")
        line["adjoint"] = adjoint_ratio(P, torch, ci)
        line["adjoint_forward_ratio"] = line["adjoint"]["ratio"]
        log(f"adjoint/forward {line['adjoint_forward_ratio']:.3f}")
    if not args.no_cpu_baseline:
        log("oracle CPU baseline ...")
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_slab)
        log(f"oracle: {line['cpu_baseline']['value']:.3e} pairs/s on "
            f"{line['cpu_baseline']['cores']} cores")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
