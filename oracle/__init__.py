"""CPU oracle for the contact-SPH hot path (test infrastructure only).

A ctypes wrapper around ``oracle.c`` (plain FP64 C, contraction off) plus
numpy conveniences.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the GPU library
never does, and this package never imports the GPU library.

State dictionaries hold numpy arrays ``x y z vx vy vz rho E m`` (float64)
and ``mat`` (int32).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-pthread"]

MAX_EOS = 8
FIELDS = ("x", "y", "z", "vx", "vy", "vz", "rho", "E", "m")


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (contraction off)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Cfg(C.Structure):
    _fields_ = [
        ("h", C.c_double),
        ("kappa", C.c_double),
        ("h_mode", C.c_int32),
        ("n_eos", C.c_int32),
        ("eos_type", C.c_int32 * MAX_EOS),
        ("eos_gamma", C.c_double * MAX_EOS),
        ("eos_pinf", C.c_double * MAX_EOS),
        ("wall", C.c_int32),
        ("search", C.c_int32),
        ("wall_x0", C.c_double),
        ("wall_v", C.c_double),
        ("cfl", C.c_double),
        ("cell_size", C.c_double),
        ("nthreads", C.c_int32),
        ("pad", C.c_int32),
        ("eos_rho0", C.c_double * MAX_EOS),
        ("eos_ca", C.c_double * MAX_EOS),
        ("eos_sa", C.c_double * MAX_EOS),
        ("periodic", C.c_int32),
        ("pad2", C.c_int32),
        ("box_lo", C.c_double * 3),
        ("box_hi", C.c_double * 3),
        ("integrator", C.c_int32),
        ("pad3", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        lp = C.POINTER(C.c_int64)
        cp = C.POINTER(Cfg)
        L.oracle_kernel_w.restype = C.c_double
        L.oracle_kernel_w.argtypes = [C.c_double, C.c_double]
        L.oracle_kernel_dw.restype = C.c_double
        L.oracle_kernel_dw.argtypes = [C.c_double, C.c_double]
        L.oracle_riemann.restype = None
        L.oracle_riemann.argtypes = [C.c_double] * 6 + [dp, dp]
        L.oracle_eos.restype = C.c_int64
        L.oracle_eos.argtypes = [cp, C.c_int64, dp, dp, dp, dp, dp, ip, dp, dp]
        L.oracle_init_energy.restype = None
        L.oracle_init_energy.argtypes = [cp, C.c_int64, dp, dp, dp, dp, dp, ip, dp]
        L.oracle_grid.restype = C.c_int
        L.oracle_grid.argtypes = [C.c_int64, dp, dp, dp, C.c_double, dp, ip]
        L.oracle_bin.restype = C.c_int
        L.oracle_bin.argtypes = [C.c_int64, dp, dp, dp, C.c_double, dp, ip, C.c_int32, ip, lp,
                                 lp, lp, C.c_int64]
        L.oracle_neighbors.restype = C.c_int64
        L.oracle_neighbors.argtypes = [cp, C.c_int64, dp, dp, dp, dp, lp, ip, C.c_int64]
        L.oracle_rates.restype = C.c_int64
        L.oracle_rates.argtypes = [cp, C.c_int64] + [dp] * 9 + [ip, dp, C.c_double] + [dp] * 6 + [lp]
        L.oracle_rates_sample.restype = C.c_int64
        L.oracle_rates_sample.argtypes = ([cp, C.c_int64] + [dp] * 9 + [ip, dp, C.c_double, lp,
                                          C.c_int64] + [dp] * 6 + [lp])
        L.oracle_dt.restype = C.c_double
        L.oracle_dt.argtypes = [cp, C.c_int64, dp, dp, dp, dp]
        L.oracle_step.restype = C.c_int64
        L.oracle_step.argtypes = [cp, C.c_int64] + [dp] * 9 + [ip, dp, dp, C.c_double, dp, lp]
        L.oracle_totals.restype = None
        L.oracle_totals.argtypes = [C.c_int64, dp, dp, dp, dp, dp, dp]
        L.oracle_exact_sum.restype = C.c_double
        L.oracle_exact_sum.argtypes = [C.c_int64, dp]
        L.oracle_voronoi.restype = None
        L.oracle_voronoi.argtypes = [C.c_int64, dp, dp, dp, C.c_int32, dp, lp, ip, lp, lp]
        L.oracle_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], (a.dtype, a.flags)
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _l(a):
    if a is None:
        return None
    assert a.dtype == np.int64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def make_cfg(eos, h=1.5, kappa=2.0, h_mode=0, wall=None, cfl=0.3, search=0, cell_size=0.0,
             nthreads=0, periodic=0, box=None, integrator=0) -> Cfg:
    """periodic: bit mask of periodic axes (1 x, 2 y, 4 z) with box = (lo[3], hi[3]);
    integrator: 0 symplectic Euler, 1 two-stage Runge-Kutta."""
    c = Cfg()
    c.h, c.kappa, c.h_mode = h, kappa, h_mode
    c.n_eos = len(eos)
    for k, e in enumerate(eos):
        # (type, gamma, p_inf) or, Mie-Grueneisen, (2, Gamma, 0, rho0, c_a, s_a)
        t, g, pinf = e[:3]
        c.eos_type[k], c.eos_gamma[k], c.eos_pinf[k] = int(t), float(g), float(pinf)
        if len(e) > 3:
            c.eos_rho0[k], c.eos_ca[k], c.eos_sa[k] = (float(v) for v in e[3:6])
    if wall is not None:
        c.wall, c.wall_x0, c.wall_v = 1, float(wall[0]), float(wall[1])
    c.cfl, c.search, c.cell_size, c.nthreads = cfl, search, cell_size, nthreads
    c.periodic = int(periodic)
    c.integrator = int(integrator)
    if box is not None:
        for a in range(3):
            c.box_lo[a], c.box_hi[a] = float(box[0][a]), float(box[1][a])
    return c


def cfg_for(w, search=0, nthreads=0, **over) -> Cfg:
    kw = dict(eos=w.eos, h=w.h, kappa=w.kappa, wall=w.wall, cfl=w.cfl, search=search,
              cell_size=w.cell_size, nthreads=nthreads, periodic=w.periodic, box=w.box)
    kw.update(over)
    return make_cfg(**kw)


def kernel_w(r: float, H: float) -> float:
    return float(lib().oracle_kernel_w(r, H))


def kernel_dw(r: float, H: float) -> float:
    return float(lib().oracle_kernel_dw(r, H))


def riemann(ZL, ZR, PL, PR, vL, vR):
    vs, ps = C.c_double(), C.c_double()
    lib().oracle_riemann(ZL, ZR, PL, PR, vL, vR, C.byref(vs), C.byref(ps))
    return vs.value, ps.value


def init_energy(cfg: Cfg, rho, p, vx, vy, vz, mat) -> np.ndarray:
    E = np.empty_like(rho)
    lib().oracle_init_energy(C.byref(cfg), rho.shape[0], _d(rho), _d(p), _d(vx), _d(vy),
                             _d(vz), _i(mat), _d(E))
    return E


def state_from(w, cfg: Optional[Cfg] = None) -> Dict[str, np.ndarray]:
    """FP64 state dict of a workload, E from the oracle's EOS inverse."""
    cfg = cfg or cfg_for(w)
    s = {k: np.ascontiguousarray(getattr(w, k), dtype=np.float64)
         for k in ("x", "y", "z", "vx", "vy", "vz", "rho", "m")}
    s["mat"] = np.ascontiguousarray(w.mat, dtype=np.int32)
    s["E"] = init_energy(cfg, s["rho"], np.ascontiguousarray(w.p, np.float64), s["vx"], s["vy"],
                         s["vz"], s["mat"])
    return s


def eos(cfg: Cfg, s):
    n = s["rho"].shape[0]
    P = np.empty(n)
    c = np.empty(n)
    bad = lib().oracle_eos(C.byref(cfg), n, _d(s["rho"]), _d(s["E"]), _d(s["vx"]), _d(s["vy"]),
                           _d(s["vz"]), _i(s["mat"]), _d(P), _d(c))
    return P, c, int(bad)


def grid(x, y, z, D):
    origin = np.zeros(3)
    dims = np.zeros(3, np.int32)
    rc = lib().oracle_grid(x.shape[0], _d(x), _d(y), _d(z), D, _d(origin), _i(dims))
    if rc != 0:
        raise ValueError("empty particle set")
    return origin, dims


def bin(x, y, z, D, origin=None, dims=None, key_mode=0):
    """Cell triples, keys, stable cell order and cell ranges (linear cells)."""
    if origin is None:
        origin, dims = grid(x, y, z, D)
    n = x.shape[0]
    cell = np.empty((n, 3), np.int32)
    key = np.empty(n, np.int64)
    perm = np.empty(n, np.int64)
    if key_mode == 1:
        bits = int(np.ceil(np.log2(max(int(dims.max()), 1)))) if int(dims.max()) > 1 else 0
        ncell = 1 << (3 * bits)
    else:
        ncell = int(dims[0]) * int(dims[1]) * int(dims[2])
    cs = np.empty(ncell + 1, np.int64)
    rc = lib().oracle_bin(n, _d(x), _d(y), _d(z), D, _d(np.ascontiguousarray(origin)),
                          _i(np.ascontiguousarray(dims, np.int32)), key_mode, _i(cell), _l(key),
                          _l(perm), _l(cs), ncell)
    if rc != 0:
        raise MemoryError
    return dict(origin=origin, dims=dims, cell=cell, key=key, perm=perm, cell_start=cs,
                ncell=ncell)


def neighbors(cfg: Cfg, x, y, z, d=None):
    n = x.shape[0]
    off = np.zeros(n + 1, np.int64)
    nnz = lib().oracle_neighbors(C.byref(cfg), n, _d(x), _d(y), _d(z), _d(d), _l(off), None, 0)
    if nnz < 0:
        raise MemoryError
    idx = np.empty(max(nnz, 1), np.int32)
    lib().oracle_neighbors(C.byref(cfg), n, _d(x), _d(y), _d(z), _d(d), _l(off), _i(idx), nnz)
    return off, idx[:nnz]


def rates(cfg: Cfg, s, t: float = 0.0, d=None):
    n = s["x"].shape[0]
    out = {k: np.empty(n) for k in ("drho", "dvx", "dvy", "dvz", "dE", "signal")}
    cnt = np.empty(n, np.int64)
    bad = lib().oracle_rates(C.byref(cfg), n, *[_d(s[k]) for k in FIELDS], _i(s["mat"]), _d(d),
                             t, _d(out["drho"]), _d(out["dvx"]), _d(out["dvy"]), _d(out["dvz"]),
                             _d(out["dE"]), _d(out["signal"]), _l(cnt))
    if bad < 0:
        raise MemoryError
    out["nbr_count"] = cnt
    out["nonphys"] = int(bad)
    return out


def rates_sample(cfg: Cfg, s, sample, t: float = 0.0, d=None):
    """Rates of the particles listed in ``sample`` (cell-list search recommended)."""
    sample = np.ascontiguousarray(sample, np.int64)
    k = sample.shape[0]
    n = s["x"].shape[0]
    out = {kk: np.empty(k) for kk in ("drho", "dvx", "dvy", "dvz", "dE", "signal")}
    cnt = np.empty(k, np.int64)
    bad = lib().oracle_rates_sample(C.byref(cfg), n, *[_d(s[kk]) for kk in FIELDS],
                                    _i(s["mat"]), _d(d), t, _l(sample), k, _d(out["drho"]),
                                    _d(out["dvx"]), _d(out["dvy"]), _d(out["dvz"]), _d(out["dE"]),
                                    _d(out["signal"]), _l(cnt))
    if bad < 0:
        raise MemoryError
    out["nbr_count"] = cnt
    return out


def dt(cfg: Cfg, signal, d=None, rho=None, drho=None) -> float:
    """cfl * min_i min(h_i/s_i, rho_i/|drho_i|) (density part only when rho, drho are given)."""
    return float(lib().oracle_dt(C.byref(cfg), signal.shape[0], _d(signal), _d(d), _d(rho),
                                 _d(drho)))


def step(cfg: Cfg, s, t: float = 0.0, dt_in: float = 0.0, d=None):
    """One step on a copy of ``s``; returns (new_state, t_new, dt_used, nbr_count)."""
    s2 = {k: v.copy() for k, v in s.items()}
    n = s2["x"].shape[0]
    tt = C.c_double(t)
    dtu = C.c_double(0.0)
    cnt = np.empty(n, np.int64)
    bad = lib().oracle_step(C.byref(cfg), n, *[_d(s2[k]) for k in FIELDS], _i(s2["mat"]),
                            _d(d), C.byref(tt), dt_in, C.byref(dtu), _l(cnt))
    if bad < 0:
        raise MemoryError
    return s2, tt.value, dtu.value, cnt


def totals(s) -> np.ndarray:
    out = np.empty(5)
    lib().oracle_totals(s["m"].shape[0], _d(s["m"]), _d(s["vx"]), _d(s["vy"]), _d(s["vz"]),
                        _d(s["E"]), _d(out))
    return out


def exact_sum(v) -> float:
    v = np.ascontiguousarray(v, np.float64)
    return float(lib().oracle_exact_sum(v.shape[0], _d(v)))


def voronoi(x, y, z, sites, nbr_count=None):
    n = x.shape[0]
    sites = np.ascontiguousarray(sites, np.float64).reshape(-1, 3)
    K = sites.shape[0]
    owner = np.empty(n, np.int32)
    sp = np.empty(K, np.int64)
    spairs = np.empty(K, np.int64)
    nc = None if nbr_count is None else np.ascontiguousarray(nbr_count, np.int64)
    lib().oracle_voronoi(n, _d(x), _d(y), _d(z), K, _d(sites.reshape(-1)), _l(nc), _i(owner),
                         _l(sp), _l(spairs))
    return owner, sp, spairs
