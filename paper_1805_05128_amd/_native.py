"""ctypes declarations of libcsph (the C ABI in include/csph.h).

Loading fails loudly when the HIP library has not been built: there is no
CPU fallback anywhere in this package.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcsph.so")

CSPH_OK, CSPH_EINVAL, CSPH_ECAPACITY, CSPH_EDEVICE, CSPH_ENONPHYS = 0, 1, 2, 3, 4
CSPH_MAX_EOS = 8
CSPH_EOS_IDEAL, CSPH_EOS_STIFFENED, CSPH_EOS_MIE_GRUNEISEN = 0, 1, 2
CSPH_FP64, CSPH_MIXED = 0, 1
CSPH_H_FIXED, CSPH_H_PAIR = 0, 1
CSPH_KEY_LINEAR, CSPH_KEY_MORTON = 0, 1
CSPH_INT_EULER, CSPH_INT_RK2 = 0, 1

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)
_up = C.POINTER(C.c_uint32)


class CsphEos(C.Structure):
    _fields_ = [("type", C.c_int32), ("pad", C.c_int32), ("gamma", C.c_double),
                ("p_inf", C.c_double), ("rho0", C.c_double), ("c_a", C.c_double),
                ("s_a", C.c_double)]


class CsphParams(C.Structure):
    _fields_ = [
        ("precision", C.c_int32), ("h_mode", C.c_int32),
        ("h", C.c_double), ("kappa", C.c_double), ("cell_size", C.c_double),
        ("cfl", C.c_double),
        ("n_eos", C.c_int32), ("wall", C.c_int32),
        ("wall_x0", C.c_double), ("wall_v", C.c_double),
        ("eos", CsphEos * CSPH_MAX_EOS),
        ("reorder", C.c_int32), ("key_mode", C.c_int32), ("check_nonphys", C.c_int32),
        ("periodic", C.c_int32), ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
        ("integrator", C.c_int32), ("pad2", C.c_int32),
    ]


class CsphState(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, _dp) for k in
                                      ("x", "y", "z", "vx", "vy", "vz", "rho", "E", "m")] + [
        ("mat", _ip), ("d", _dp), ("id", _lp)]


class CsphGrid(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("cell", C.c_double), ("inv_cell", C.c_double),
                ("dims", C.c_int32 * 3), ("reach", C.c_int32), ("ncell", C.c_int64),
                ("key_mode", C.c_int32), ("pad", C.c_int32), ("nkey", C.c_int64)]


class CsphRatesOut(C.Structure):
    _fields_ = [(k, _dp) for k in ("drho", "dvx", "dvy", "dvz", "dE")]


class CsphGrad(C.Structure):
    _fields_ = [(k, _dp) for k in ("x", "y", "z", "vx", "vy", "vz", "rho", "E")]


PROF_GROUPS = ("bin", "pack", "rates", "integrate", "voronoi", "reorder", "neighbors", "adjoint",
               "balance")


class CsphProfile(C.Structure):
    _fields_ = [("launches", C.c_int64 * len(PROF_GROUPS)), ("ms", C.c_double * len(PROF_GROUPS))]


class CsphBalanceParams(C.Structure):
    _fields_ = [("sigma", C.c_double), ("theta", C.c_double), ("gamma", C.c_double),
                ("dsh", C.c_double)]


_lib = None


class CsphError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


class NonPhysicalState(CsphError):
    """CSPH_ENONPHYS: the call wrote its outputs, but some particle's state was non-physical
    (negative or NaN squared sound speed; its sound speed was taken as 0)."""


def load():
    """The loaded libcsph (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1805_05128_amd.build` (no CPU fallback exists)")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    sz = C.c_size_t
    szp = C.POINTER(C.c_size_t)
    L.csph_status_string.restype = C.c_char_p
    L.csph_status_string.argtypes = [C.c_int32]
    L.csph_last_error.restype = C.c_char_p
    L.csph_last_error.argtypes = []
    L.csph_version.restype = C.c_char_p
    L.csph_version.argtypes = []
    L.csph_workspace_size.restype = sz
    L.csph_workspace_size.argtypes = [C.c_int64, C.c_int64, C.POINTER(CsphParams)]
    L.csph_grid_build.restype = C.c_int32
    L.csph_grid_build.argtypes = [_dp, _dp, _dp, C.c_int64, C.POINTER(CsphParams), _dp,
                                  C.POINTER(CsphGrid), vp, sz, vp]
    L.csph_bin.restype = C.c_int32
    L.csph_bin.argtypes = [_dp, _dp, _dp, C.c_int64, C.POINTER(CsphGrid), _up, _ip, _ip,
                           C.c_int64, vp, sz, szp, vp]
    L.csph_neighbors.restype = C.c_int32
    L.csph_neighbors.argtypes = [C.POINTER(CsphState), C.POINTER(CsphParams), _lp, _ip,
                                 C.c_int64, _lp, vp, sz, szp, vp]
    L.csph_rates.restype = C.c_int32
    L.csph_rates.argtypes = [C.POINTER(CsphState), C.POINTER(CsphParams), C.c_double,
                             CsphRatesOut, _dp, _ip, _lp, vp, sz, szp, vp]
    L.csph_step.restype = C.c_int32
    L.csph_step.argtypes = [C.POINTER(CsphState), C.POINTER(CsphState), C.POINTER(CsphParams),
                            _dp, C.c_double, _dp, _dp, _ip, _lp, vp, sz, szp, vp]
    L.csph_step_voronoi.restype = C.c_int32
    L.csph_step_voronoi.argtypes = [C.POINTER(CsphState), C.POINTER(CsphState),
                                    C.POINTER(CsphParams), _dp, C.c_double, _dp, _dp, _ip, _lp,
                                    _dp, C.c_int32, _ip, _lp, _lp, vp, sz, szp, vp]
    L.csph_step_static.restype = C.c_int32
    L.csph_step_static.argtypes = [C.POINTER(CsphState), C.POINTER(CsphState),
                                   C.POINTER(CsphParams), _dp, C.c_double, _dp, _dp, _ip, _lp,
                                   vp]
    L.csph_step_mesh.restype = C.c_int32
    L.csph_step_mesh.argtypes = [C.POINTER(CsphState), C.POINTER(CsphState),
                                 C.POINTER(CsphParams), C.POINTER(CsphGrid), _dp, C.c_double,
                                 _dp, _dp, _ip, _lp, _lp, vp, sz, szp, vp]
    L.voronoi_assign.restype = C.c_int32
    L.voronoi_assign.argtypes = [_dp, _dp, _dp, C.c_int64, _dp, C.c_int32, _ip, _ip, _lp, _lp,
                                 vp]
    L.csph_init_energy.restype = C.c_int32
    L.csph_init_energy.argtypes = [_dp, _dp, _dp, _dp, _dp, _ip, C.c_int64,
                                   C.POINTER(CsphParams), _dp, vp]
    L.csph_rates_vjp.restype = C.c_int32
    L.csph_rates_vjp.argtypes = [C.POINTER(CsphState), C.POINTER(CsphParams), C.c_double,
                                 CsphRatesOut, CsphGrad, _dp, vp, sz, szp, vp]
    L.csph_step_vjp.restype = C.c_int32
    L.csph_step_vjp.argtypes = [C.POINTER(CsphState), C.POINTER(CsphParams), C.c_double,
                                C.c_double, CsphGrad, CsphGrad, _dp, vp, sz, szp, vp]
    L.csph_step_vjp_cfl.restype = C.c_int32
    L.csph_step_vjp_cfl.argtypes = [C.POINTER(CsphState), C.POINTER(CsphParams), C.c_double,
                                    CsphGrad, CsphGrad, _dp, _dp, vp, sz, szp, vp]
    L.csph_init_energy_vjp.restype = C.c_int32
    L.csph_init_energy_vjp.argtypes = [_dp, _dp, _dp, _dp, _dp, _ip, C.c_int64,
                                       C.POINTER(CsphParams), _dp, _dp, _dp, _dp, _dp, _dp, vp,
                                       sz, szp, vp]
    L.csph_vlist_build.restype = C.c_int32
    L.csph_vlist_build.argtypes = [C.POINTER(CsphState), C.POINTER(CsphState),
                                   C.POINTER(CsphParams), _dp, C.c_double, C.c_int32, _ip, _ip,
                                   _dp, vp, C.POINTER(C.c_int32), vp, sz, szp, vp]
    L.csph_step_vlist.restype = C.c_int32
    L.csph_step_vlist.argtypes = [C.POINTER(CsphState), C.POINTER(CsphParams), _dp, C.c_double,
                                  _dp, _dp, _ip, _lp, _ip, _ip, C.c_int32, _dp, vp, vp, sz,
                                  szp, vp]
    L.csph_balance_workspace_size.restype = sz
    L.csph_balance_workspace_size.argtypes = [C.c_int32]
    L.csph_balance_stats.restype = C.c_int32
    L.csph_balance_stats.argtypes = [_dp, _dp, _dp, C.c_int64, _ip, _ip, _dp, C.c_int32,
                                     C.c_double, _lp, _lp, _dp, _up, vp, sz, szp, vp]
    L.csph_balance_move.restype = C.c_int32
    L.csph_balance_move.argtypes = [_dp, C.c_int32, _lp, _dp, _up, C.POINTER(CsphBalanceParams),
                                    _dp, _dp, vp]
    L.csph_profile_enable.restype = C.c_int32
    L.csph_profile_enable.argtypes = [C.c_int32]
    L.csph_profile_groups.restype = C.c_int32
    L.csph_profile_groups.argtypes = [C.c_uint32]
    L.csph_profile_read.restype = C.c_int32
    L.csph_profile_read.argtypes = [C.POINTER(CsphProfile)]
    _lib = L
    return L


def check(status: int, where: str):
    if status != CSPH_OK:
        L = load()
        msg = (L.csph_last_error() or b"").decode() or L.csph_status_string(status).decode()
        cls = NonPhysicalState if status == CSPH_ENONPHYS else CsphError
        raise cls(status, where, msg)
