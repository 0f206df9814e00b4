"""torch.autograd.Function over a CSPH rollout with the hand-written adjoint.

The forward runs ``nsteps`` steps (particle order kept) from initial
velocities and adiabatic indices, storing the state every ``every`` steps
and recording the time-step sequence.  The backward walks the segments in
reverse: it restores a segment's checkpoint, recomputes the segment's
states with the recorded time steps (bit-identical to the forward), then
applies csph_step_vjp step by step and finally the VJP of the initial
energy E0 = e(rho, p; gamma) + |v0|^2/2 when the rollout starts from
(rho, p) (a window that starts from (rho, E) holds E fixed).  By default
the time steps are held fixed (replayed), i.e. the gradient is that of the
map at the recorded dt sequence; with ``cfl_adjoint`` each step's VJP is
csph_step_vjp_cfl, which differentiates the CFL step as well.  The start
time of every step is recorded too:
with the piston, the segments are replayed from their own start times and
each step's VJP places the wall where the step did.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import torch

from . import api as A

STATE8 = A.GRAD_FIELDS


def _fresh_like(s: A.State) -> A.State:
    """Uninitialised evolving fields for a step's output; mass, material and sizes shared."""
    t = {k: (v if k == "m" else torch.empty_like(v)) for k, v in s.t.items()}
    return A.State(t, s.mat, s.d, None)


def _with_gamma(params: A.Params, gamma: List[float]) -> A.Params:
    """The run's parameters with each material's gamma (Grueneisen Gamma for a Mie-Grueneisen
    material) replaced; its other constants kept."""
    eos = [(e[0], float(g)) + tuple(e[2:]) for e, g in zip(params.eos, gamma)]
    return dataclasses.replace(params, eos=eos, reorder=False, precision="fp64")


class CSPHRollout(torch.autograd.Function):
    """(vx0, vy0, vz0, gamma) -> final state (x, y, z, vx, vy, vz, rho, E).

    ``base`` holds the device tensors x, y, z, rho, m, mat (and, in pair-h
    mode, the particle sizes d, held fixed) of the initial state and either p (the initial energy is then E0 = e(rho, p; gamma) +
    |v0|^2/2, differentiated) or E (a window that starts from a state of a
    longer run: E is held fixed, so the gradient is the partial derivative
    at fixed specific total energy); ``params`` the run parameters (its
    gammas are replaced by the ``gamma`` tensor); ``dts``, if given, is the
    list of time steps to use instead of the CFL rule; ``t0`` the start time
    (the piston's position); ``cfl_adjoint`` differentiates the CFL time steps
    too (csph_step_vjp_cfl; only without ``dts``), so that the gradient is that
    of the rollout as run rather than of the map at its recorded steps.  After
    the call, ``info['dts']`` holds the dt sequence and ``info['forward_s']``
    the forward wall time.
    """

    @staticmethod
    def forward(ctx, vx0, vy0, vz0, gamma, base: Dict[str, torch.Tensor], params: A.Params,
                nsteps: int, every: int, dts: Optional[List[float]], info: dict,
                t0: float = 0.0, cfl_adjoint: bool = False):
        import time
        torch.cuda.synchronize()
        tic = time.perf_counter()
        if cfl_adjoint and (dts is not None or not params.cfl > 0.0):
            raise ValueError("cfl_adjoint needs the CFL rule (cfl > 0) and no dts")
        pg = _with_gamma(params, gamma.detach().cpu().tolist())
        if "p" in base:
            E0 = A.csph_init_energy(base["rho"], base["p"], vx0, vy0, vz0, base["mat"], pg)
        else:
            E0 = base["E"].clone()
        st = A.State({"x": base["x"].clone(), "y": base["y"].clone(), "z": base["z"].clone(),
                      "vx": vx0.detach().clone(), "vy": vy0.detach().clone(),
                      "vz": vz0.detach().clone(), "rho": base["rho"].clone(), "E": E0,
                      "m": base["m"]}, base["mat"], base.get("d"))
        sc = A.StepScalars(vx0.device, t0=t0)
        ckpts = []
        # each step writes its dt straight into the record (sc.dt a view of one slot); the
        # start times follow on the host, t_{k+1} = t_k + dt_k, the step's own FP64 addition
        dt_rec = torch.empty(nsteps, dtype=torch.float64, device=vx0.device)
        replay = dataclasses.replace(pg, cfl=0.0)
        # every step writes a fresh state, so a checkpoint is the state itself (no copies)
        for k in range(nsteps):
            if k % every == 0:
                ckpts.append(st)
            nxt = _fresh_like(st)
            sc.dt = dt_rec[k:k + 1]
            if dts is None:
                A.csph_step(st, pg, sc, s_out=nxt, totals=False)
            else:
                A.csph_step(st, replay, sc, s_out=nxt, dt_in=float(dts[k]), totals=False)
            st = nxt
        dt_list = dt_rec.cpu().tolist()
        t_list, tk = [], float(t0)
        for dt in dt_list:
            t_list.append(tk)
            tk = tk + dt
        if nsteps and tk != float(sc.t.item()):
            raise RuntimeError("the recorded start times do not reproduce the device's time")
        torch.cuda.synchronize()
        info["dts"] = dt_list
        info["forward_s"] = time.perf_counter() - tic
        ctx.ckpts = ckpts
        ctx.dts = dt_list
        ctx.ts = t_list
        ctx.cfl_adjoint = cfl_adjoint
        ctx.params = pg
        ctx.every = every
        ctx.nsteps = nsteps
        ctx.base = base
        ctx.info = info
        ctx.save_for_backward(vx0, vy0, vz0)
        return tuple(st.t[k].clone() for k in STATE8)

    @staticmethod
    def backward(ctx, *g_final):
        import time
        torch.cuda.synchronize()
        tic = time.perf_counter()
        vx0, vy0, vz0 = ctx.saved_tensors
        dev = vx0.device
        n = vx0.shape[0]
        pg = ctx.params
        g = {k: (gf.contiguous().clone() if gf is not None else torch.zeros(n, dtype=torch.float64, device=dev))
             for k, gf in zip(STATE8, g_final)}
        g_eos = torch.zeros(2 * len(pg.eos), dtype=torch.float64, device=dev)
        replay = dataclasses.replace(pg, cfl=0.0)
        nseg = len(ctx.ckpts)
        for seg in reversed(range(nseg)):
            k0 = seg * ctx.every
            k1 = min(k0 + ctx.every, ctx.nsteps)
            # the segment's replay starts at its recorded time; t + dt then repeats the
            # forward's times bit for bit
            sc = A.StepScalars(dev, t0=ctx.ts[k0])
            # each replayed step writes a fresh state (no copies; the checkpoint is only read)
            states = [ctx.ckpts[seg]]
            for k in range(k0, k1 - 1):
                s = _fresh_like(states[-1])
                A.csph_step(states[-1], replay, sc, s_out=s, dt_in=ctx.dts[k], totals=False)
                states.append(s)
            for k in reversed(range(k0, k1)):
                if ctx.cfl_adjoint:
                    _, _, dt = A.csph_step_vjp_cfl(states[k - k0], pg, g, g_prev=g, g_eos=g_eos,
                                                   t=ctx.ts[k])
                    if dt != ctx.dts[k]:
                        raise RuntimeError(f"step {k}: the CFL step recomputed for its adjoint "
                                           f"({dt!r}) differs from the forward's ({ctx.dts[k]!r})")
                else:
                    A.csph_step_vjp(states[k - k0], pg, ctx.dts[k], g, g_prev=g, g_eos=g_eos,
                                    t=ctx.ts[k])
            states.clear()
        b = ctx.base
        if "p" in b:
            A.csph_init_energy_vjp(b["rho"], b["p"], vx0, vy0, vz0, b["mat"], pg, g["E"],
                                   g_v=(g["vx"], g["vy"], g["vz"]), g_eos=g_eos)
        torch.cuda.synchronize()
        ctx.info["backward_s"] = time.perf_counter() - tic
        return (g["vx"], g["vy"], g["vz"], g_eos[0::2].clone(), None, None, None, None, None,
                None, None, None)


def rollout(vx0, vy0, vz0, gamma, base, params, nsteps, every=10, dts=None, info=None,
            t0: float = 0.0, cfl_adjoint: bool = False):
    """Functional form of CSPHRollout.apply; returns a dict of final-state tensors.

    By default the gradient is that of the rollout at a FIXED time-step sequence: the forward records
    the CFL time steps it took (or takes ``dts``), and the backward differentiates the map
    with those steps held constant.  The dependence of the CFL step on the state and on
    gamma (through c, the closing speeds and rho/|drho/dt|) is not differentiated, so a
    finite-difference check must replay the same steps.  With ``cfl_adjoint`` the CFL steps
    are differentiated too (the forward must take them: no ``dts``), and a finite-difference
    check reruns the CFL rule."""
    info = {} if info is None else info
    out = CSPHRollout.apply(vx0, vy0, vz0, gamma, base, params, nsteps, every, dts, info, t0,
                            cfl_adjoint)
    return dict(zip(STATE8, out))
