"""C-ABI library checks that need no GPU: it loads, exports every function
include/csph.h declares, and rejects bad arguments before any device work."""
import ctypes as C
import os
import re

import pytest

import paper_1805_05128_amd as P
from paper_1805_05128_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"^[A-Za-z_][\w \*]*?\b(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


def test_library_exports_every_declared_function():
    L = N.load()
    names = header_functions()
    assert "csph_step" in names and "voronoi_assign" in names and len(names) >= 10
    for n in names:
        assert hasattr(L, n), n


def test_status_strings_and_version():
    L = N.load()
    for s in (0, 1, 2, 3, 4):
        assert L.csph_status_string(s).decode().startswith("CSPH_")
    assert b"ENONPHYS" in L.csph_status_string(N.CSPH_ENONPHYS)
    assert P.version().startswith("csph-gfx950")


def test_workspace_size_grows():
    p = P.Params()
    a = P.workspace_size(1000, 100, p)
    b = P.workspace_size(2000, 100, p)
    c = P.workspace_size(2000, 10_000, p)
    assert 0 < a < b < c
    assert b - a >= 1000 * 200  # per-particle buffers


@pytest.mark.parametrize("bad", [
    dict(eos=[(0, 1.0, 0.0)]),
    dict(eos=[(7, 1.4, 0.0)]),
    dict(eos=[]),
    dict(h=0.0),
    dict(kappa=-1.0),
    dict(precision="half"),
])
def test_invalid_params_rejected_without_device_work(bad):
    L = N.load()
    kw = dict(eos=[(0, 1.4, 0.0)])
    prec = bad.pop("precision", None)
    kw.update(bad)
    p = P.Params(**kw).c()
    if prec is not None:
        p.precision = 9
    st = L.csph_init_energy(None, None, None, None, None, None, 0, C.byref(p), None, None)
    assert st == N.CSPH_EINVAL
    assert L.csph_last_error()


def test_invalid_arguments_rejected():
    L = N.load()
    p = P.Params().c()
    assert L.voronoi_assign(None, None, None, 10, None, 4, None, None, None, None,
                            None) == N.CSPH_EINVAL
    assert L.voronoi_assign(None, None, None, 0, None, 0, None, None, None, None,
                            None) == N.CSPH_EINVAL
    s = N.CsphState()
    s.n = -1
    assert L.csph_rates(C.byref(s), C.byref(p), 0.0, N.CsphRatesOut(), None, None, None, None, 0,
                        None, None) == N.CSPH_EINVAL
    s.n = 5  # NULL field pointers
    assert L.csph_step(C.byref(s), C.byref(s), C.byref(p), None, 0.0, None, None, None, None,
                       None, 0, None, None) == N.CSPH_EINVAL


def test_pair_walks_reject_more_than_2_to_27_particles():
    """Pair kernels address 32-byte records with 32-bit offsets: n >= 2^27 is refused on the
    host, before any device work (the field pointers are never dereferenced)."""
    L = N.load()
    p = P.Params().c()
    s = N.CsphState()
    s.n = 1 << 27
    for f in ("x", "y", "z", "vx", "vy", "vz", "rho", "E", "m"):
        setattr(s, f, C.cast(C.c_void_p(4096), C.POINTER(C.c_double)))
    out = N.CsphRatesOut()
    assert L.csph_rates(C.byref(s), C.byref(p), 0.0, out, None, None, None, None, 0,
                        None, None) == N.CSPH_EINVAL
    assert b"2^27" in L.csph_last_error()
    assert L.csph_step(C.byref(s), C.byref(s), C.byref(p), None, 0.0, None, None, None, None,
                       None, 0, None, None) == N.CSPH_EINVAL
    assert b"2^27" in L.csph_last_error()


def test_vlist_build_rejects_misaligned_list_storage():
    """List chunks are stored as 16-byte vectors: a misaligned vl_idx is refused on the host,
    before any device work (pointers are never dereferenced)."""
    L = N.load()
    p = P.Params().c()
    a, b = N.CsphState(), N.CsphState()
    for st, base in ((a, 4096), (b, 8192)):
        st.n = 100
        for k, f in enumerate(("x", "y", "z", "vx", "vy", "vz", "rho", "E", "m")):
            setattr(st, f, C.cast(C.c_void_p(base + 1024 * k), C.POINTER(C.c_double)))
    dev = lambda addr, t: C.cast(C.c_void_p(addr), C.POINTER(t))
    st = L.csph_vlist_build(C.byref(a), C.byref(b), C.byref(p), None, 0.3, 64,
                            dev(65536, C.c_int32), dev(131072 + 4, C.c_int32),
                            dev(262144, C.c_double), None, None, None, 0, None, None)
    assert st == N.CSPH_EINVAL
    assert b"16-byte aligned" in L.csph_last_error()


def _fake_state(base, n=100):
    s = N.CsphState()
    s.n = n
    for k, f in enumerate(("x", "y", "z", "vx", "vy", "vz", "rho", "E", "m")):
        setattr(s, f, C.cast(C.c_void_p(base + 1024 * k), C.POINTER(C.c_double)))
    return s


def test_wall_steps_need_the_time():
    """With the piston wall the step places the plane at t: a NULL t is refused on the host,
    before any device work, by the per-step search and by the Verlet-list step."""
    L = N.load()
    p = P.Params(wall=(0.0, 2.0)).c()
    a, b = _fake_state(4096), _fake_state(65536)
    st = L.csph_step(C.byref(a), C.byref(b), C.byref(p), None, 0.0, None, None, None, None,
                     None, 0, None, None)
    assert st == N.CSPH_EINVAL and b"needs t" in L.csph_last_error()
    dev = lambda addr, t: C.cast(C.c_void_p(addr), C.POINTER(t))
    st = L.csph_step_vlist(C.byref(a), C.byref(p), None, 0.0, None, None, None, None,
                           dev(1 << 20, C.c_int32), dev(1 << 21, C.c_int32), 64,
                           dev(1 << 22, C.c_double), None, None, 0, None, None)
    assert st == N.CSPH_EINVAL and b"needs t" in L.csph_last_error()


def test_key_mode_checked():
    L = N.load()
    p = P.Params().c()
    p.key_mode = 7
    st = L.csph_init_energy(None, None, None, None, None, None, 0, C.byref(p), None, None)
    assert st == N.CSPH_EINVAL and b"key_mode" in L.csph_last_error()
    # a grid whose key space does not match its dims and key mode
    g = N.CsphGrid()
    g.inv_cell, g.cell = 1.0, 1.0
    g.dims[0], g.dims[1], g.dims[2] = 5, 3, 2
    g.ncell = 30
    g.key_mode = N.CSPH_KEY_MORTON
    g.nkey = 30  # the Morton key space of 5 x 3 x 2 cells is 2^(3*3) = 512
    dev = lambda addr, t: C.cast(C.c_void_p(addr), C.POINTER(t))
    x = dev(4096, C.c_double)
    st = L.csph_bin(x, x, x, 10, C.byref(g), None, dev(8192, C.c_int32),
                    dev(16384, C.c_int32), 1000, None, 0, None, None)
    assert st == N.CSPH_EINVAL and b"nkey" in L.csph_last_error()
    g.nkey = 512
    st = L.csph_bin(x, x, x, 10, C.byref(g), None, dev(8192, C.c_int32),
                    dev(16384, C.c_int32), 100, None, 0, None, None)
    assert st == N.CSPH_ECAPACITY and b"513" in L.csph_last_error()


def test_list_step_needs_its_control_block():
    """csph_step_vlist checks the lists' exactness bound on the device, in their control
    block: a missing or misaligned block is refused on the host, before any device work."""
    L = N.load()
    p = P.Params().c()
    a = _fake_state(4096)
    dev = lambda addr, t: C.cast(C.c_void_p(addr), C.POINTER(t))
    for ctl in (None, C.c_void_p(1 << 23 | 4)):
        st = L.csph_step_vlist(C.byref(a), C.byref(p), dev(1 << 24, C.c_double), 0.0, None, None,
                               None, None, dev(1 << 20, C.c_int32), dev(1 << 21, C.c_int32), 64,
                               dev(1 << 22, C.c_double), ctl, None, 0, None, None)
        assert st == N.CSPH_EINVAL and b"ctl" in L.csph_last_error()


def test_periodic_params_checked_on_the_host():
    """Periodic boundaries: an unknown axis mask, an empty box, a periodic wall axis, and the
    calls that do not take periodic boundaries (Verlet lists) are refused before any device
    work; so is the adjoint in pair-h mode without the sizes d."""
    L = N.load()
    box = ((0.0, 0.0, 0.0), (10.0, 10.0, 10.0))
    for kw, msg in ((dict(periodic=9, box=box), b"periodic mask"),
                    (dict(periodic=2, box=((0.0, 5.0, 0.0), (10.0, 5.0, 10.0))), b"box_hi > box_lo"),
                    (dict(periodic=1, box=box, wall=(0.0, 1.0)), b"wall's axis")):
        p = P.Params(**kw).c()
        st = L.csph_init_energy(None, None, None, None, None, None, 0, C.byref(p), None, None)
        assert st == N.CSPH_EINVAL and msg in L.csph_last_error(), kw
    p = P.Params(periodic=6, box=box, wall=(0.0, 1.0)).c()  # periodic across the wall: valid
    assert L.csph_init_energy(None, None, None, None, None, None, 0, C.byref(p), None,
                              None) == N.CSPH_OK
    p = P.Params(periodic=7, box=box).c()
    a, b = _fake_state(4096), _fake_state(65536)
    dev = lambda addr, t: C.cast(C.c_void_p(addr), C.POINTER(t))
    st = L.csph_vlist_build(C.byref(a), C.byref(b), C.byref(p), None, 0.3, 64,
                            dev(1 << 20, C.c_int32), dev(1 << 21, C.c_int32),
                            dev(1 << 22, C.c_double), None, None, None, 0, None, None)
    assert st == N.CSPH_EINVAL and b"periodic" in L.csph_last_error()
    st = L.csph_step_vlist(C.byref(a), C.byref(p), dev(1 << 24, C.c_double), 0.0, None, None,
                           None, None, dev(1 << 20, C.c_int32), dev(1 << 21, C.c_int32), 64,
                           dev(1 << 22, C.c_double), C.c_void_p(1 << 23), None, 0, None, None)
    assert st == N.CSPH_EINVAL and b"periodic" in L.csph_last_error()
    g = N.CsphGrad(*[dev((1 << 25) + 1024 * k, C.c_double) for k in range(8)])
    p = P.Params(periodic=7, box=box, h_mode="pair").c()  # the adjoint in pair-h mode needs d
    st = L.csph_step_vjp(C.byref(a), C.byref(p), 0.0, 0.1, g, g, None, None, 0, None, None)
    assert st == N.CSPH_EINVAL and b"particle size array d" in L.csph_last_error()


def test_integrator_checked_on_the_host():
    """An unknown integrator, and the two-stage Runge-Kutta step where only the Euler step is
    taken (Verlet-list steps, the CFL step's adjoint), are refused before any device work; the
    workspace of a Runge-Kutta step is larger."""
    L = N.load()
    p = P.Params().c()
    p.integrator = 5
    st = L.csph_init_energy(None, None, None, None, None, None, 0, C.byref(p), None, None)
    assert st == N.CSPH_EINVAL and b"integrator" in L.csph_last_error()
    p = P.Params(integrator="rk2").c()
    a = _fake_state(4096)
    dev = lambda addr, t: C.cast(C.c_void_p(addr), C.POINTER(t))
    st = L.csph_step_vlist(C.byref(a), C.byref(p), dev(1 << 24, C.c_double), 0.0, None, None,
                           None, None, dev(1 << 20, C.c_int32), dev(1 << 21, C.c_int32), 64,
                           dev(1 << 22, C.c_double), C.c_void_p(1 << 23), None, 0, None, None)
    assert st == N.CSPH_EINVAL and b"Euler" in L.csph_last_error()
    g = N.CsphGrad(*[dev((1 << 25) + 1024 * k, C.c_double) for k in range(8)])
    st = L.csph_step_vjp_cfl(C.byref(a), C.byref(p), 0.0, g, g, None, None, None, 0, None, None)
    assert st == N.CSPH_EINVAL and b"Euler" in L.csph_last_error()
    assert P.workspace_size(1000, 100, P.Params(integrator="rk2")) > \
        P.workspace_size(1000, 100, P.Params()) + 1000 * 150


def test_step_mesh_checked_on_the_host():
    """csph_step_mesh refuses, before any device work: no mesh, pair-h mode, check_nonphys
    (it would wait), and a mesh whose reach does not cover the support."""
    L = N.load()
    a, b = _fake_state(4096), _fake_state(65536)
    g = N.CsphGrid()
    g.cell, g.inv_cell = 1.0, 1.0
    g.dims[0] = g.dims[1] = g.dims[2] = 4
    g.ncell, g.reach = 64, 3
    call = lambda p, mesh: L.csph_step_mesh(C.byref(a), C.byref(b), C.byref(p), mesh, None,
                                            0.1, None, None, None, None, None, None, 0, None,
                                            None)
    assert call(P.Params(cfl=0.0).c(), None) == N.CSPH_EINVAL
    assert b"mesh" in L.csph_last_error()
    a.d = b.d = C.cast(C.c_void_p(1 << 26), C.POINTER(C.c_double))  # pair-h mode needs d
    assert call(P.Params(cfl=0.0, h_mode="pair").c(), C.byref(g)) == N.CSPH_EINVAL
    assert b"fixed-h" in L.csph_last_error()
    a.d = b.d = None
    assert call(P.Params(cfl=0.0, check_nonphys=True).c(), C.byref(g)) == N.CSPH_EINVAL
    assert b"check_nonphys" in L.csph_last_error()
    g.reach = 2
    assert call(P.Params(cfl=0.0).c(), C.byref(g)) == N.CSPH_EINVAL
    assert b"reach" in L.csph_last_error()
    g.reach, g.ncell = 3, 65
    assert call(P.Params(cfl=0.0).c(), C.byref(g)) == N.CSPH_EINVAL
    assert b"ncell" in L.csph_last_error()
