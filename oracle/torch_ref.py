"""Differentiable CPU reference of the CSPH rates and step (test infrastructure only).

Plain PyTorch CPU FP64 operations over an explicit pair list, written from
the same equations as ``oracle.c`` (sec. 4.1, eqs. SPH:Conti, SPH:Pulse,
SPH:Energy, acoustic pairwise Riemann solver, Wendland C2 kernel) so that
``torch.autograd`` supplies exact reference gradients for the hand-written
GPU adjoint.  Pair lists come from the C oracle's brute-force neighbour
sets.  The time step dt is an input (frozen), fixed-h mode only, no wall.

Only the tests may import this module.
"""
from __future__ import annotations

import math
from typing import Dict, Sequence, Tuple

import numpy as np
import torch

import oracle as O

FIELDS8 = ("x", "y", "z", "vx", "vy", "vz", "rho", "E")


def pairs_of(cfg, s) -> Tuple[torch.Tensor, torch.Tensor]:
    """Directed pair list (i, j), j in N(i), from the oracle's neighbour sets."""
    off, idx = O.neighbors(cfg, np.ascontiguousarray(s["x"]), np.ascontiguousarray(s["y"]),
                           np.ascontiguousarray(s["z"]))
    i = np.repeat(np.arange(len(off) - 1), np.diff(off))
    return torch.as_tensor(i, dtype=torch.long), torch.as_tensor(idx.astype(np.int64))


def eos_torch(rho, E, vx, vy, vz, mat, eos_type: Sequence[int], gamma, pinf):
    """P and c from e = E - |v|^2/2 (ideal or stiffened gas), per-material gamma/p_inf tensors."""
    e = E - 0.5 * ((vx * vx + vy * vy) + vz * vz)
    g = gamma[mat]
    pi = pinf[mat]
    stiff = torch.as_tensor([t == 1 for t in eos_type], dtype=torch.bool)[mat]
    P = torch.where(stiff, (g - 1.0) * rho * e - g * pi, (g - 1.0) * rho * e)
    c2 = torch.where(stiff, g * (P + pi) / rho, g * P / rho)
    c = torch.sqrt(torch.clamp(c2, min=0.0))
    return P, c


def init_energy_torch(rho, p, vx, vy, vz, mat, eos_type, gamma, pinf):
    g = gamma[mat]
    pi = pinf[mat]
    stiff = torch.as_tensor([t == 1 for t in eos_type], dtype=torch.bool)[mat]
    e = torch.where(stiff, (p + g * pi) / ((g - 1.0) * rho), p / ((g - 1.0) * rho))
    return e + 0.5 * ((vx * vx + vy * vy) + vz * vz)


def rates_torch(st: Dict[str, torch.Tensor], m, mat, eos_type, gamma, pinf, pairs, H: float):
    """(drho, dvx, dvy, dvz, dE) of every particle for the directed pair list."""
    x, y, z, vx, vy, vz, rho, E = (st[k] for k in FIELDS8)
    P, c = eos_torch(rho, E, vx, vy, vz, mat, eos_type, gamma, pinf)
    Z = rho * c
    V = m / rho
    i, j = pairs
    dx, dy, dz = x[j] - x[i], y[j] - y[i], z[j] - z[i]
    r2 = (dx * dx + dy * dy) + dz * dz
    nz = r2 > 0
    r = torch.sqrt(torch.where(nz, r2, torch.ones_like(r2)))
    ex, ey, ez = dx / r, dy / r, dz / r
    q = r / H
    a = 1.0 - q
    dW = torch.where(nz, -(210.0 / (math.pi * H ** 4)) * q * a ** 3, torch.zeros_like(r))
    vL = (vx[i] * ex + vy[i] * ey) + vz[i] * ez
    vR = (vx[j] * ex + vy[j] * ey) + vz[j] * ez
    Zi, Zj, Pi, Pj = Z[i], Z[j], P[i], P[j]
    S = Zi + Zj
    Ss = torch.where(S != 0, S, torch.ones_like(S))
    vs = torch.where(S != 0, ((Zi * vL + Zj * vR) + (Pi - Pj)) / Ss, 0.5 * (vL + vR))
    ps = torch.where(S != 0, ((Zj * Pi + Zi * Pj) + Zi * Zj * (vL - vR)) / Ss, 0.5 * (Pi + Pj))
    w = V[j] * dW
    n = x.shape[0]
    z0 = torch.zeros(n, dtype=x.dtype)
    s_rho = z0.index_add(0, i, w * (vL - vs))
    f = w * ps
    s_vx = z0.index_add(0, i, f * ex)
    s_vy = z0.index_add(0, i, f * ey)
    s_vz = z0.index_add(0, i, f * ez)
    s_E = z0.index_add(0, i, f * vs)
    return (-2.0 * rho * s_rho, (2.0 / rho) * s_vx, (2.0 / rho) * s_vy, (2.0 / rho) * s_vz,
            (2.0 / rho) * s_E)


def step_torch(st, m, mat, eos_type, gamma, pinf, pairs, H: float, dt: float):
    """Symplectic Euler with frozen dt: v, E, rho += dt rates, then r += dt v_new."""
    drho, dvx, dvy, dvz, dE = rates_torch(st, m, mat, eos_type, gamma, pinf, pairs, H)
    vx = st["vx"] + dt * dvx
    vy = st["vy"] + dt * dvy
    vz = st["vz"] + dt * dvz
    return {"x": st["x"] + dt * vx, "y": st["y"] + dt * vy, "z": st["z"] + dt * vz,
            "vx": vx, "vy": vy, "vz": vz, "rho": st["rho"] + dt * drho, "E": st["E"] + dt * dE}


def to_torch(s) -> Dict[str, torch.Tensor]:
    return {k: torch.as_tensor(np.asarray(s[k], np.float64)) for k in FIELDS8}


def to_numpy(st, m, mat) -> dict:
    out = {k: st[k].detach().numpy().copy() for k in FIELDS8}
    out["m"] = m.detach().numpy().copy()
    out["mat"] = mat.numpy().astype(np.int32)
    return out
