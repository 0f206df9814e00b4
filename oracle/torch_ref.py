"""Differentiable CPU reference of the CSPH rates and step (test infrastructure only).

Plain PyTorch CPU FP64 operations over an explicit pair list, written from
the same equations as ``oracle.c`` (sec. 4.1, eqs. SPH:Conti, SPH:Pulse,
SPH:Energy, acoustic pairwise Riemann solver, Wendland C2 kernel) so that
``torch.autograd`` supplies exact reference gradients for the hand-written
GPU adjoint.  Pair lists come from the C oracle's brute-force neighbour
sets; with the piston (the rigid wall of sec. 7.1) the mirror pairs come from
a brute-force test of the reflected positions written as the oracle writes it,
and the step reflects the particles that cross the plane.  The materials are
ideal gas, stiffened gas, or Mie-Grueneisen (eqs. mie_gruneisen_eos,
mie_gruneisen_reference, with the sound speed the oracle derives from them).
The time step dt is an input (frozen); in pair-h mode the particle sizes d are
constants of the map.

Only the tests may import this module.
"""
from __future__ import annotations

import math
from typing import Dict, Sequence, Tuple

import numpy as np
import torch

import oracle as O

FIELDS8 = ("x", "y", "z", "vx", "vy", "vz", "rho", "E")


def _support(H, pair_h, i, j):
    """The support of each pair: H (fixed-h mode), or kappa (d_i + d_j)/2 with pair_h =
    (kappa, d) (pair-h mode, d held fixed)."""
    if pair_h is None:
        return H
    kappa, d = pair_h
    d = torch.as_tensor(np.asarray(d, np.float64))
    return kappa * (0.5 * (d[i] + d[j]))


def pairs_of(cfg, s):
    """Directed pair list (i, j), j in N(i), from the oracle's neighbour sets.  With periodic
    axes, (i, j, shift): shift[p, a] = k_a L_a of the image through which j is i's partner (the
    offset is (x_j - x_i) - k L, as the oracle forms it); with each period above twice the
    support that image is the one nearest i, k_a = round((x_j - x_i) / L_a)."""
    d = s.get("d") if cfg.h_mode == 1 else None
    off, idx = O.neighbors(cfg, np.ascontiguousarray(s["x"]), np.ascontiguousarray(s["y"]),
                           np.ascontiguousarray(s["z"]),
                           None if d is None else np.ascontiguousarray(d, np.float64))
    i = np.repeat(np.arange(len(off) - 1), np.diff(off))
    j = idx.astype(np.int64)
    ti, tj = torch.as_tensor(i, dtype=torch.long), torch.as_tensor(j)
    if not cfg.periodic:
        return ti, tj
    shift = np.zeros((len(i), 3))
    for a, k in enumerate(("x", "y", "z")):
        if (cfg.periodic >> a) & 1:
            L = cfg.box_hi[a] - cfg.box_lo[a]
            v = np.asarray(s[k], np.float64)
            shift[:, a] = np.round((v[j] - v[i]) / L) * L
    return ti, tj, torch.as_tensor(shift)


def mirror_pairs_of(s, H: float, xw: float, box=None, periodic: int = 0, pair_h=None):
    """Directed mirror pairs (i, j), j = i included: the reflected position of j,
    (2 xw - x_j, y_j, z_j), within the support of i; brute force over all j, the squared
    distance formed as the oracle forms it (((dx dx) + (dy dy)) + dz dz, dx = xg - x_i).
    With periodic axes y and z (the wall's axis x is never periodic), the image of the
    reflected j nearest i, and (i, j, shift) as from ``pairs_of``.  pair_h = (kappa, d): the
    support kappa (d_i + d_j)/2 of each pair instead of H."""
    x, y, z = (np.asarray(s[k], np.float64) for k in ("x", "y", "z"))
    xg = 2.0 * xw - x
    dx = xg[None, :] - x[:, None]
    d = [dx, y[None, :] - y[:, None], z[None, :] - z[:, None]]
    sh = [np.zeros_like(dx) for _ in range(3)]
    for a in (1, 2):
        if (periodic >> a) & 1:
            L = box[1][a] - box[0][a]
            sh[a] = np.round(d[a] / L) * L
            d[a] = d[a] - sh[a]
    r2 = ((d[0] * d[0]) + (d[1] * d[1])) + (d[2] * d[2])
    if pair_h is None:
        i, j = np.nonzero(r2 < H * H)
    else:
        kappa, dd = pair_h
        dd = np.asarray(dd, np.float64)
        Hij = kappa * (0.5 * (dd[:, None] + dd[None, :]))
        i, j = np.nonzero(r2 < Hij * Hij)
    ti, tj = torch.as_tensor(i.astype(np.int64)), torch.as_tensor(j.astype(np.int64))
    if not periodic:
        return ti, tj
    return ti, tj, torch.as_tensor(np.stack([sh[a][i, j] for a in range(3)], axis=1))


def _materials(eos_type, mat):
    """Per-particle type codes and Mie-Grueneisen constants (rho0, c_a, s_a).  ``eos_type``
    holds, per material, its type code or its whole tuple (type, gamma, p_inf[, rho0, c_a,
    s_a]); materials of other types take the harmless constants (1, 1, 0)."""
    types, mg = [], []
    for e in eos_type:
        t = int(e[0]) if isinstance(e, (tuple, list)) else int(e)
        types.append(t)
        mg.append(tuple(float(v) for v in e[3:6]) if t == 2 else (1.0, 1.0, 0.0))
    ty = torch.as_tensor(types, dtype=torch.int64)[mat]
    k = torch.as_tensor(mg, dtype=torch.float64)[mat]
    return ty, k[:, 0], k[:, 1], k[:, 2]


def _mg_reference(rho, rho0, ca, sa):
    """Reference curves of the linear u_s - u_p Hugoniot at x = rho0/rho: (P_r, e_r, D, x, eta)
    with D = 1 - s_a (1 - x)."""
    x = rho0 / rho
    eta = 1.0 - x
    D = 1.0 - sa * eta
    D2 = D * D
    return rho0 * ca * ca * eta / D2, 0.5 * ca * ca * eta * eta / D2, D, x, eta


def eos_torch(rho, E, vx, vy, vz, mat, eos_type: Sequence, gamma, pinf):
    """P and c from e = E - |v|^2/2, per-material gamma (Gamma) / p_inf tensors."""
    e = E - 0.5 * ((vx * vx + vy * vy) + vz * vz)
    g = gamma[mat]
    pi = pinf[mat]
    ty, rho0, ca, sa = _materials(eos_type, mat)
    P = torch.where(ty == 1, (g - 1.0) * rho * e - g * pi, (g - 1.0) * rho * e)
    c2 = torch.where(ty == 1, g * (P + pi) / rho, g * P / rho)
    if bool((ty == 2).any()):
        # P = P_r + Gamma rho (e - e_r); c^2 = (dP/drho)_e + (P/rho^2)(dP/de)_rho
        Pr, er, D, x, eta = _mg_reference(rho, rho0, ca, sa)
        D3 = D * D * D
        Pm = Pr + g * rho * (e - er)
        dPr = ca * ca * x * x * (1.0 + sa * eta) / D3
        rder = ca * ca * eta * x / D3
        c2m = dPr + g * (e - er) - g * rder + g * Pm / rho
        c2m = torch.where(D > 0.0, c2m, torch.full_like(c2m, -1.0))
        P = torch.where(ty == 2, Pm, P)
        c2 = torch.where(ty == 2, c2m, c2)
    c = torch.sqrt(torch.clamp(c2, min=0.0))
    return P, c


def init_energy_torch(rho, p, vx, vy, vz, mat, eos_type, gamma, pinf):
    g = gamma[mat]
    pi = pinf[mat]
    ty, rho0, ca, sa = _materials(eos_type, mat)
    # the gas forms divide by gamma - 1: a Mie-Grueneisen particle (whose Gamma may be 1)
    # evaluates them, unused, at gamma = 2, keeping their gradients finite
    gg = torch.where(ty == 2, torch.full_like(g, 2.0), g)
    e = torch.where(ty == 1, (p + gg * pi) / ((gg - 1.0) * rho), p / ((gg - 1.0) * rho))
    if bool((ty == 2).any()):
        Pr, er, _, _, _ = _mg_reference(rho, rho0, ca, sa)
        e = torch.where(ty == 2, er + (p - Pr) / (g * rho), e)
    return e + 0.5 * ((vx * vx + vy * vy) + vz * vz)


def _pair_sums(x, y, z, vx, vy, vz, P, Z, V, i, j, xj, vxj, H: float, shift=None):
    """Per-pair terms of i's sums for partners j whose position's x and velocity's x are
    ``xj`` and ``vxj`` (the particle's own, or its mirror image's), through the periodic
    images ``shift`` (k L per pair and axis) when given."""
    dx, dy, dz = xj - x[i], y[j] - y[i], z[j] - z[i]
    if shift is not None:
        dx, dy, dz = dx - shift[:, 0], dy - shift[:, 1], dz - shift[:, 2]
    r2 = (dx * dx + dy * dy) + dz * dz
    nz = r2 > 0
    r = torch.sqrt(torch.where(nz, r2, torch.ones_like(r2)))
    ex, ey, ez = dx / r, dy / r, dz / r
    q = r / H
    a = 1.0 - q
    dW = torch.where(nz, -(210.0 / (math.pi * H ** 4)) * q * a ** 3, torch.zeros_like(r))
    vL = (vx[i] * ex + vy[i] * ey) + vz[i] * ez
    vR = (vxj * ex + vy[j] * ey) + vz[j] * ez
    Zi, Zj, Pi, Pj = Z[i], Z[j], P[i], P[j]
    S = Zi + Zj
    Ss = torch.where(S != 0, S, torch.ones_like(S))
    vs = torch.where(S != 0, ((Zi * vL + Zj * vR) + (Pi - Pj)) / Ss, 0.5 * (vL + vR))
    ps = torch.where(S != 0, ((Zj * Pi + Zi * Pj) + Zi * Zj * (vL - vR)) / Ss, 0.5 * (Pi + Pj))
    w = V[j] * dW
    f = w * ps
    return w * (vL - vs), f * ex, f * ey, f * ez, f * vs


def rates_torch(st: Dict[str, torch.Tensor], m, mat, eos_type, gamma, pinf, pairs, H: float,
                mirror=None, wall=None, pair_h=None):
    """(drho, dvx, dvy, dvz, dE) of every particle for the directed pair list, plus, with the
    piston wall = (x_w, v_w) at the evaluation time, the directed mirror pairs: j's mirror image
    at 2 x_w - x_j with x-velocity 2 v_w - vx_j and j's other fields.  pair_h = (kappa, d):
    pair-h mode, each pair's support kappa (d_i + d_j)/2 (d constant)."""
    x, y, z, vx, vy, vz, rho, E = (st[k] for k in FIELDS8)
    P, c = eos_torch(rho, E, vx, vy, vz, mat, eos_type, gamma, pinf)
    Z = rho * c
    V = m / rho
    n = x.shape[0]
    z0 = torch.zeros(n, dtype=x.dtype)
    sums = [z0] * 5
    i, j = pairs[0], pairs[1]
    shift = pairs[2] if len(pairs) > 2 else None
    for k, t in enumerate(_pair_sums(x, y, z, vx, vy, vz, P, Z, V, i, j, x[j], vx[j],
                                     _support(H, pair_h, i, j), shift)):
        sums[k] = sums[k].index_add(0, i, t)
    if mirror is not None:
        xw, vw = wall
        i, j = mirror[0], mirror[1]
        terms = _pair_sums(x, y, z, vx, vy, vz, P, Z, V, i, j, 2.0 * xw - x[j],
                           2.0 * vw - vx[j], _support(H, pair_h, i, j),
                           mirror[2] if len(mirror) > 2 else None)
        for k, t in enumerate(terms):
            sums[k] = sums[k].index_add(0, i, t)
    s_rho, s_vx, s_vy, s_vz, s_E = sums
    return (-2.0 * rho * s_rho, (2.0 / rho) * s_vx, (2.0 / rho) * s_vy, (2.0 / rho) * s_vz,
            (2.0 / rho) * s_E)


def cfl_dt_torch(st, m, mat, eos_type, gamma, pinf, pairs, H: float, cfl: float, h: float,
                 mirror=None, wall=None, pair_h=None):
    """The CFL time step as a differentiable function of the state and EOS parameters:
    dt = cfl min_i min(h_i / s_i, rho_i / |drho_i|), h_i = h (fixed) or d_i (pair h), the
    signal speed s_i = max(c_i, max over partners (mirror partners included) of
    max(c_i, c_j) + max(0, v_L - v_R)) with v_L - v_R = (v_i - v_j).e, e pointing from i to
    j (wall = (x_w, v_w) at the evaluation time).  The minimum and the maxima pass their
    gradients to the particle and the partner that attain them."""
    x, y, z, vx, vy, vz, rho, E = (st[k] for k in FIELDS8)
    P, c = eos_torch(rho, E, vx, vy, vz, mat, eos_type, gamma, pinf)
    drho = rates_torch(st, m, mat, eos_type, gamma, pinf, pairs, H, mirror=mirror, wall=wall,
                       pair_h=pair_h)[0]
    sig = c
    lists = [(pairs, x, vx, pairs[2] if len(pairs) > 2 else None)]
    if mirror is not None:
        xw, vw = wall
        lists.append((mirror, 2.0 * xw - x, 2.0 * vw - vx, mirror[2] if len(mirror) > 2 else None))
    for pr, xs, vxs, shift in lists:
        i, j = pr[0], pr[1]
        dx, dy, dz = xs[j] - x[i], y[j] - y[i], z[j] - z[i]
        if shift is not None:
            dx, dy, dz = dx - shift[:, 0], dy - shift[:, 1], dz - shift[:, 2]
        r = torch.sqrt((dx * dx + dy * dy) + dz * dz)
        closing = ((vx[i] - vxs[j]) * dx + (vy[i] - vy[j]) * dy + (vz[i] - vz[j]) * dz) / r
        sp = torch.maximum(c[i], c[j]) + torch.clamp(closing, min=0.0)
        sig = sig.scatter_reduce(0, i, sp, reduce="amax", include_self=True)
    hi = h if pair_h is None else torch.as_tensor(np.asarray(pair_h[1], np.float64))
    tau = torch.minimum(hi / sig, rho / torch.abs(drho))
    return cfl * torch.min(tau)


def step_torch(st, m, mat, eos_type, gamma, pinf, pairs, H: float, dt: float, mirror=None,
               wall=None, t: float = 0.0, box=None, periodic: int = 0, pair_h=None):
    """Symplectic Euler with frozen dt: v, E, rho += dt rates, then r += dt v_new.  With the
    piston wall = (x_w0, v_w): mirror pairs at x_w(t), and a particle whose new x lies behind
    x_w(t + dt) is reflected (x <- 2 x_w - x, v_x <- 2 v_w - v_x, E changed by the kinetic
    energy difference); which particles reflect is decided on the values (a fixed branch for
    the gradient).  Periodic axes (bit mask, box = (lo, hi)): a new position at or above hi
    moves down by the period, one below lo up by it, after the reflection."""
    w_now = None if wall is None else (wall[0] + wall[1] * t, wall[1])
    drho, dvx, dvy, dvz, dE = rates_torch(st, m, mat, eos_type, gamma, pinf, pairs, H,
                                          mirror=mirror, wall=w_now, pair_h=pair_h)
    vx = st["vx"] + dt * dvx
    vy = st["vy"] + dt * dvy
    vz = st["vz"] + dt * dvz
    x = st["x"] + dt * vx
    E = st["E"] + dt * dE
    if wall is not None:
        xw = wall[0] + wall[1] * (t + dt)
        behind = (x < xw).detach()
        vr = 2.0 * wall[1] - vx
        E = torch.where(behind, E + 0.5 * ((vr * vr) - (vx * vx)), E)
        vx = torch.where(behind, vr, vx)
        x = torch.where(behind, 2.0 * xw - x, x)
    pos = [x, st["y"] + dt * vy, st["z"] + dt * vz]
    for a in range(3):
        if (periodic >> a) & 1:
            lo, hi = float(box[0][a]), float(box[1][a])
            L = hi - lo
            p = pos[a]
            up, down = (p >= hi).detach(), (p < lo).detach()
            pos[a] = torch.where(up, p - L, torch.where(down, p + L, p))
    return {"x": pos[0], "y": pos[1], "z": pos[2],
            "vx": vx, "vy": vy, "vz": vz, "rho": st["rho"] + dt * drho, "E": E}


def step_rk2_torch(st, m, mat, eos_type, gamma, pinf, pairs_at, H: float, dt: float,
                   mirror_at=None, wall=None, t: float = 0.0, box=None, periodic: int = 0,
                   pair_h=None):
    """The two-stage Runge-Kutta step with frozen dt, as the oracle takes it (Shu and Osher's
    convex form): U1 = U + dt F(U, t), r1 = r + dt v; U' = U/2 + (U1 + dt F(U1, t + dt))/2,
    r' = r/2 + (r1 + dt v1)/2; the second evaluation sees r1 wrapped into a periodic box (and
    the piston at x_w(t + dt)); then the reflection and the wrap of the Euler step.
    ``pairs_at(pos)`` and ``mirror_at(pos, x_w)`` give the pair lists of a set of positions
    (numpy arrays x, y, z), taken at the values (fixed for the gradient)."""
    def wrap(pos):
        out = list(pos)
        for a in range(3):
            if (periodic >> a) & 1:
                lo, hi = float(box[0][a]), float(box[1][a])
                L = hi - lo
                p = out[a]
                up, down = (p >= hi).detach(), (p < lo).detach()
                out[a] = torch.where(up, p - L, torch.where(down, p + L, p))
        return out

    def npos(q):
        return {k: v.detach().numpy() for k, v in zip(("x", "y", "z"), q)}

    def rates_at(u, pos, tt):
        xw = None if wall is None else wall[0] + wall[1] * tt
        mir = None if wall is None else mirror_at(npos(pos), xw)
        su = {"x": pos[0], "y": pos[1], "z": pos[2], "vx": u["vx"], "vy": u["vy"],
              "vz": u["vz"], "rho": u["rho"], "E": u["E"]}
        return rates_torch(su, m, mat, eos_type, gamma, pinf, pairs_at(npos(pos)), H,
                           mirror=mir, wall=None if wall is None else (xw, wall[1]),
                           pair_h=pair_h)

    r0 = [st["x"], st["y"], st["z"]]
    f0 = rates_at(st, r0, t)
    u1 = {"vx": st["vx"] + dt * f0[1], "vy": st["vy"] + dt * f0[2], "vz": st["vz"] + dt * f0[3],
          "E": st["E"] + dt * f0[4], "rho": st["rho"] + dt * f0[0]}
    r1 = [st[k] + dt * st["v" + k] for k in ("x", "y", "z")]
    f1 = rates_at(u1, wrap(r1), t + dt)
    vx = 0.5 * st["vx"] + 0.5 * (u1["vx"] + dt * f1[1])
    vy = 0.5 * st["vy"] + 0.5 * (u1["vy"] + dt * f1[2])
    vz = 0.5 * st["vz"] + 0.5 * (u1["vz"] + dt * f1[3])
    E = 0.5 * st["E"] + 0.5 * (u1["E"] + dt * f1[4])
    rho = 0.5 * st["rho"] + 0.5 * (u1["rho"] + dt * f1[0])
    pos = [0.5 * r0[a] + 0.5 * (r1[a] + dt * u1["v" + k]) for a, k in enumerate("xyz")]
    x = pos[0]
    if wall is not None:
        xw = wall[0] + wall[1] * (t + dt)
        behind = (x < xw).detach()
        vr = 2.0 * wall[1] - vx
        E = torch.where(behind, E + 0.5 * ((vr * vr) - (vx * vx)), E)
        vx = torch.where(behind, vr, vx)
        x = torch.where(behind, 2.0 * xw - x, x)
    pos = wrap([x, pos[1], pos[2]])
    return {"x": pos[0], "y": pos[1], "z": pos[2], "vx": vx, "vy": vy, "vz": vz, "rho": rho,
            "E": E}


def to_torch(s) -> Dict[str, torch.Tensor]:
    return {k: torch.as_tensor(np.asarray(s[k], np.float64)) for k in FIELDS8}


def to_numpy(st, m, mat) -> dict:
    out = {k: st[k].detach().numpy().copy() for k in FIELDS8}
    out["m"] = m.detach().numpy().copy()
    out["mat"] = mat.numpy().astype(np.int32)
    return out
