"""Seeded synthetic particle sets for the contact-SPH hot path.

This module only lays particles out and assigns the primitive state the
workload recipes state (density, pressure, velocity, material id). It holds
none of the method's arithmetic: no equation of state, no energy, no kernel,
no binning. Both the GPU library's tests and the CPU oracle draw their
inputs from here, so that the two sides see identical bits.

Geometry conventions (all workloads):
  * lattice sites at (i+1/2, j+1/2, k+1/2) with spacing 1 (plus a shift);
  * seeded jitter uniform in [-0.01, 0.01] per coordinate (1 % of spacing);
  * particle mass = density x spacing^3 (one lattice cell per particle);
  * smoothing length h = 1.5 with support kappa*h, kappa = 2 (support 3).

Random streams: ``numpy.random.default_rng(SeedSequence(seed).spawn(4))``
gives [jitter, voids/centres, Voronoi sites, finite-difference directions].
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

EOS_IDEAL = 0
EOS_STIFFENED = 1
EOS_MIE_GRUNEISEN = 2
# Mie-Grueneisen materials of sec. 5 as (type, Gamma, 0, rho0 [g/cc], c_a [km/s], s_a)
MG_LEAD = (EOS_MIE_GRUNEISEN, 1.7, 0.0, 11.35, 2.58, 1.26)
MG_ALUMINIUM = (EOS_MIE_GRUNEISEN, 1.5, 0.0, 1.593, 3.0, 1.85)

JITTER = 0.01
H_SMOOTH = 1.5
KAPPA = 2.0


@dataclass
class Workload:
    """One synthetic particle set plus the run parameters of its recipe."""

    name: str
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    rho: np.ndarray
    p: np.ndarray
    m: np.ndarray
    mat: np.ndarray
    # (type, gamma, p_inf) per material id
    eos: List[Tuple[int, float, float]]
    h: float = H_SMOOTH
    kappa: float = KAPPA
    cell_size: float = H_SMOOTH * KAPPA
    wall: Optional[Tuple[float, float]] = None  # (x0, velocity) of a +x-facing piston
    periodic: int = 0  # bit mask of periodic axes (1 x, 2 y, 4 z) ...
    box: Optional[Tuple[Tuple[float, float, float], Tuple[float, float, float]]] = None  # ... box
    cfl: float = 0.3
    steps: int = 1
    sites: Optional[np.ndarray] = None  # (K, 3) Voronoi generators
    fd_dirs: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def _streams(seed: int):
    ss = np.random.SeedSequence(seed).spawn(4)
    return [np.random.default_rng(s) for s in ss]


def lattice(nx: int, ny: int, nz: int, shift=(0.0, 0.0, 0.0)):
    """Sites (i+1/2, j+1/2, k+1/2) + shift, x fastest."""
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x = i.reshape(-1).astype(np.float64) + 0.5 + shift[0]
    y = j.reshape(-1).astype(np.float64) + 0.5 + shift[1]
    z = k.reshape(-1).astype(np.float64) + 0.5 + shift[2]
    return x, y, z


def jitter(rng, *coords, amp=JITTER):
    out = []
    for c in coords:
        out.append(c + rng.uniform(-amp, amp, size=c.shape))
    return out


def _base(x, y, z, rho, p, mat=None, v=(0.0, 0.0, 0.0)):
    n = x.shape[0]
    rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), (n,)).copy()
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), (n,)).copy()
    vx = np.full(n, v[0], dtype=np.float64)
    vy = np.full(n, v[1], dtype=np.float64)
    vz = np.full(n, v[2], dtype=np.float64)
    if mat is None:
        mat = np.zeros(n, dtype=np.int32)
    m = rho * 1.0  # density x spacing^3
    return dict(x=x, y=y, z=z, vx=vx, vy=vy, vz=vz, rho=rho, p=p, m=m, mat=np.asarray(mat, np.int32))


def sod(nside: int, seed: int, split: float, name: str, steps: int = 1) -> Workload:
    """Cubic jittered lattice with a two-state split at x = split (ideal gas 1.4)."""
    r = _streams(seed)
    x, y, z = lattice(nside, nside, nside)
    x, y, z = jitter(r[0], x, y, z)
    left = x < split
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    st = _base(x, y, z, rho, p)
    return Workload(name=name, eos=[(EOS_IDEAL, 1.4, 0.0)], steps=steps, **st)


def config0() -> Workload:
    """4096 particles, 16^3 jittered lattice, Sod split at x=8, one rate evaluation + one step, FP64."""
    return sod(16, 1, 8.0, "sod16_4096", steps=1)


def config1() -> Workload:
    """Plate impact: 128x128x32 target at rest struck by a 64x64x16 projectile at v_z=-5.

    Stiffened gas gamma=3, p_inf=1/3 (sound speed ~1 at rho=1, p=1e-3).
    The projectile's bottom layer sits at z=34.5, one support radius above the
    target's top layer (z=31.5). 128*128*32 + 64*64*16 = 589 824 particles.
    """
    r = _streams(2)
    tx, ty, tz = lattice(128, 128, 32)
    px, py, pz = lattice(64, 64, 16, shift=(32.0, 32.0, 34.0))
    x = np.concatenate([tx, px])
    y = np.concatenate([ty, py])
    z = np.concatenate([tz, pz])
    x, y, z = jitter(r[0], x, y, z)
    st = _base(x, y, z, 1.0, 1e-3)
    st["vz"][tx.shape[0]:] = -5.0
    return Workload(name="plate_impact_589824", eos=[(EOS_STIFFENED, 3.0, 1.0 / 3.0)],
                    steps=200, **st)


def carve_voids(nside: int, rng, radius: float = 5.0, porosity: float = 0.30):
    """Boolean keep-mask over the nside^3 lattice after seeded spherical voids.

    Void centres are drawn uniformly in [0, nside)^3 one at a time; every site
    closer than ``radius`` to a centre is removed; drawing stops once the
    removed fraction reaches ``porosity``.
    """
    keep = np.ones((nside, nside, nside), dtype=bool)  # [k, j, i]
    total = nside ** 3
    removed = 0
    target = porosity * total
    rr = int(np.ceil(radius)) + 1
    r2 = radius * radius
    while removed < target:
        c = rng.uniform(0.0, float(nside), size=3)
        lo = np.maximum(np.floor(c - rr).astype(int), 0)
        hi = np.minimum(np.floor(c + rr).astype(int) + 1, nside)
        ii = np.arange(lo[0], hi[0]) + 0.5 - c[0]
        jj = np.arange(lo[1], hi[1]) + 0.5 - c[1]
        kk = np.arange(lo[2], hi[2]) + 0.5 - c[2]
        d2 = (kk[:, None, None] ** 2 + jj[None, :, None] ** 2) + ii[None, None, :] ** 2
        sub = keep[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        hit = (d2 < r2) & sub
        removed += int(hit.sum())
        sub[hit] = False
    return keep.reshape(-1)


def config2(nside: int = 256, voids: bool = True) -> Workload:
    """Porous sample shock: nside^3 lattice with 30 % spherical voids (radius 5), piston at x=0 moving +x at 2.

    Ideal gas 1.4, rho=1, p=1, at rest; 64 Voronoi sites uniform in [0, nside)^3.
    ``voids=False`` gives the void-free twin of the same lattice.
    """
    r = _streams(3)
    x, y, z = lattice(nside, nside, nside)
    if voids:
        keep = carve_voids(nside, r[1])
        x, y, z = x[keep], y[keep], z[keep]
    x, y, z = jitter(r[0], x, y, z)
    st = _base(x, y, z, 1.0, 1.0)
    sites = r[2].uniform(0.0, float(nside), size=(64, 3))
    name = f"porous_shock_{nside}cubed" + ("" if voids else "_voidfree")
    return Workload(name=name, eos=[(EOS_IDEAL, 1.4, 0.0)], wall=(0.0, 2.0), steps=100,
                    sites=sites, **st)


def config3(nside: int = 64) -> Workload:
    """Adjoint run: 64^3 Sod split at x=32, 100 steps, checkpoint every 10.

    Courant number 0.1 (the recipe states none): 100 steps then reach t ~ 7,
    before free-surface particles of the open cube enter the rho -> 0 regime
    where the map becomes too ill-conditioned for finite differences.
    """
    w = sod(nside, 4, nside / 2.0, f"adjoint_sod_{nside}cubed", steps=100)
    w.cfl = 0.1
    w.cell_size = 1.0  # unit mesh cells (the neighbour sets do not depend on the mesh)
    r = _streams(4)
    w.fd_dirs = r[3].standard_normal((32, 3 * w.n + 1))
    return w


def config4(nx: int = 400, ny: int = 400, nz: int = 200) -> Workload:
    """Two-body collision: B (rho 1, ideal 1.4, v_z=+4) below A (rho 10, stiffened 3, v_z=-4)."""
    r = _streams(5)
    bx, by, bz = lattice(nx, ny, nz)
    ax, ay, az = lattice(nx, ny, nz, shift=(0.0, 0.0, float(nz) + 2.0))
    nb = bx.shape[0]
    x = np.concatenate([bx, ax])
    y = np.concatenate([by, ay])
    z = np.concatenate([bz, az])
    x, y, z = jitter(r[0], x, y, z)
    rho = np.concatenate([np.full(nb, 1.0), np.full(nb, 10.0)])
    p = np.concatenate([np.full(nb, 1.0 / 1.4), np.full(nb, 1e-3)])
    mat = np.concatenate([np.zeros(nb, np.int32), np.ones(nb, np.int32)])
    st = _base(x, y, z, rho, p, mat=mat)
    st["vz"][:nb] = 4.0
    st["vz"][nb:] = -4.0
    return Workload(name=f"collision_{2 * nb}", steps=50,
                    eos=[(EOS_IDEAL, 1.4, 0.0), (EOS_STIFFENED, 3.0, 10.0 / 3.0 - 1e-3)], **st)


def mg_plates(nx: int = 256, ny: int = 256, nz: int = 48, gap: float = 2.0,
              v_impact: float = 0.5, seed: int = 9) -> Workload:
    """Aluminium plate moving at v_z = -v_impact onto a lead plate of the same lattice size,
    Mie-Grueneisen materials of sec. 5 (g/cc, km/s, GPa), both at the reference state
    (P = 0); ``gap`` lattice spacings between the facing layers."""
    r = _streams(seed)
    lx, ly, lz = lattice(nx, ny, nz)
    ax, ay, az = lattice(nx, ny, nz, shift=(0.0, 0.0, float(nz) - 1.0 + gap))
    x, y, z = jitter(r[0], np.concatenate([lx, ax]), np.concatenate([ly, ay]),
                     np.concatenate([lz, az]))
    nl = lx.shape[0]
    mat = np.concatenate([np.zeros(nl, np.int32), np.ones(nl, np.int32)])
    rho = np.where(mat == 0, MG_LEAD[3], MG_ALUMINIUM[3]).astype(np.float64)
    st = _base(x, y, z, rho, 0.0, mat=mat)
    st["vz"][nl:] = -v_impact
    return Workload(name=f"mg_plates_{2 * nl}", eos=[MG_LEAD, MG_ALUMINIUM], steps=20, **st)


def random_cloud(n: int, seed: int, box: float = 8.0, vmax: float = 0.3,
                 rho_range=(0.5, 2.0), p_range=(0.2, 2.0), n_mat: int = 1) -> Workload:
    """Uniform random particles in [0, box)^3 with random primitive state (edge-case tests)."""
    r = _streams(seed)
    x = r[0].uniform(0.0, box, n)
    y = r[0].uniform(0.0, box, n)
    z = r[0].uniform(0.0, box, n)
    vx = r[1].uniform(-vmax, vmax, n)
    vy = r[1].uniform(-vmax, vmax, n)
    vz = r[1].uniform(-vmax, vmax, n)
    rho = r[1].uniform(*rho_range, n)
    p = r[1].uniform(*p_range, n)
    mat = (r[2].integers(0, n_mat, n)).astype(np.int32)
    m = r[2].uniform(0.5, 1.5, n)
    eos = [(EOS_IDEAL, 1.4, 0.0), (EOS_STIFFENED, 3.0, 0.5)][:max(1, n_mat)]
    return Workload(name=f"cloud{n}_s{seed}", x=x, y=y, z=z, vx=vx, vy=vy, vz=vz, rho=rho, p=p,
                    m=m, mat=mat, eos=eos)


def jittered_block(nx: int, ny: int, nz: int, seed: int, rho=1.0, p=1.0,
                   v=(0.0, 0.0, 0.0), eos=None, amp=JITTER, shift=(0.0, 0.0, 0.0)) -> Workload:
    r = _streams(seed)
    x, y, z = lattice(nx, ny, nz, shift)
    if amp > 0:
        x, y, z = jitter(r[0], x, y, z, amp=amp)
    st = _base(x, y, z, rho, p, v=v)
    return Workload(name=f"block{nx}x{ny}x{nz}_s{seed}", eos=eos or [(EOS_IDEAL, 1.4, 0.0)], **st)


def periodic_block(nx: int, ny: int, nz: int, seed: int, periodic: int = 7, amp=JITTER,
                   rho=1.0, p=1.0, v=(0.0, 0.0, 0.0), eos=None) -> Workload:
    """Jittered lattice filling the box [0, n)^3 exactly (spacing 1, sites at i + 1/2), periodic
    along the axes of the bit mask ``periodic`` (1 x, 2 y, 4 z)."""
    w = jittered_block(nx, ny, nz, seed=seed, rho=rho, p=p, v=v, eos=eos, amp=amp)
    w.periodic = int(periodic)
    w.box = ((0.0, 0.0, 0.0), (float(nx), float(ny), float(nz)))
    w.name = f"periodic{periodic}_{nx}x{ny}x{nz}_s{seed}"
    return w


def voronoi_sites(k: int, seed: int, box) -> np.ndarray:
    r = _streams(seed)
    return r[2].uniform(0.0, 1.0, size=(k, 3)) * np.asarray(box, dtype=np.float64)


def fd_directions(count: int, dim: int, seed: int) -> np.ndarray:
    """Gaussian directions normalised to unit length (finite-difference checks)."""
    r = _streams(seed)
    d = r[3].standard_normal((count, dim))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


CONFIGS = {0: config0, 1: config1, 2: config2, 3: config3, 4: config4}
