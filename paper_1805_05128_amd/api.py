"""Python binding of libcsph: the C-ABI calls under the same names.

Only argument marshalling happens here: torch supplies device memory and
the current HIP stream, and every step of the hot path runs in the HIP
kernels behind ``include/csph.h``.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import _native as N

STATE_FIELDS = ("x", "y", "z", "vx", "vy", "vz", "rho", "E", "m")
EOS_IDEAL, EOS_STIFFENED = N.CSPH_EOS_IDEAL, N.CSPH_EOS_STIFFENED
EOS_MIE_GRUNEISEN = N.CSPH_EOS_MIE_GRUNEISEN


def _ptr(t: Optional[torch.Tensor], ctype):
    if t is None:
        return None
    return C.cast(C.c_void_p(t.data_ptr()), C.POINTER(ctype))


def _dp(t):
    if t is not None:
        assert t.dtype == torch.float64 and t.is_contiguous() and t.is_cuda, (t.dtype, t.device)
    return _ptr(t, C.c_double)


def _ip(t):
    if t is not None:
        assert t.dtype == torch.int32 and t.is_contiguous() and t.is_cuda
    return _ptr(t, C.c_int32)


def _lp(t):
    if t is not None:
        assert t.dtype == torch.int64 and t.is_contiguous() and t.is_cuda
    return _ptr(t, C.c_int64)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


@dataclass
class Params:
    """Mirror of csph_params."""

    eos: List[Tuple] = field(default_factory=lambda: [(EOS_IDEAL, 1.4, 0.0)])
    precision: str = "fp64"  # "fp64" | "mixed"
    h: float = 1.5
    kappa: float = 2.0
    h_mode: str = "fixed"  # "fixed" | "pair"
    cell_size: float = 0.0
    cfl: float = 0.3
    wall: Optional[Tuple[float, float]] = None
    reorder: bool = True
    key_mode: str = "linear"  # "linear" | "morton": keys csph_bin reports
    check_nonphys: bool = False  # csph_step: wait and raise NonPhysicalState (state written)
    periodic: int = 0  # bit mask of periodic axes (1 x, 2 y, 4 z) ...
    box: Optional[Tuple[Tuple[float, float, float], Tuple[float, float, float]]] = None  # ... box
    integrator: str = "euler"  # "euler" (symplectic Euler) | "rk2" (two-stage Runge-Kutta)

    def c(self) -> N.CsphParams:
        p = N.CsphParams()
        p.precision = N.CSPH_MIXED if self.precision == "mixed" else N.CSPH_FP64
        p.h_mode = N.CSPH_H_PAIR if self.h_mode == "pair" else N.CSPH_H_FIXED
        p.h, p.kappa, p.cell_size, p.cfl = self.h, self.kappa, self.cell_size, self.cfl
        p.n_eos = len(self.eos)
        for k, e in enumerate(self.eos):
            # (type, gamma, p_inf), or Mie-Grueneisen (EOS_MIE_GRUNEISEN, Gamma, 0, rho0, c_a, s_a)
            t, g, pinf = e[:3]
            p.eos[k].type, p.eos[k].gamma, p.eos[k].p_inf = int(t), float(g), float(pinf)
            if len(e) > 3:
                p.eos[k].rho0, p.eos[k].c_a, p.eos[k].s_a = (float(v) for v in e[3:6])
        if self.wall is not None:
            p.wall, p.wall_x0, p.wall_v = 1, float(self.wall[0]), float(self.wall[1])
        p.reorder = 1 if self.reorder else 0
        p.key_mode = N.CSPH_KEY_MORTON if self.key_mode == "morton" else N.CSPH_KEY_LINEAR
        p.check_nonphys = 1 if self.check_nonphys else 0
        p.periodic = int(self.periodic)
        p.integrator = N.CSPH_INT_RK2 if self.integrator == "rk2" else N.CSPH_INT_EULER
        if self.box is not None:
            for a in range(3):
                p.box_lo[a], p.box_hi[a] = float(self.box[0][a]), float(self.box[1][a])
        return p

    @classmethod
    def from_workload(cls, w, **over) -> "Params":
        kw = dict(eos=list(w.eos), h=w.h, kappa=w.kappa, cell_size=w.cell_size, cfl=w.cfl,
                  wall=w.wall, periodic=getattr(w, "periodic", 0), box=getattr(w, "box", None))
        kw.update(over)
        return cls(**kw)


class State:
    """Device particle state (FP64 SoA) mirroring csph_state."""

    def __init__(self, tensors: Dict[str, torch.Tensor], mat: Optional[torch.Tensor] = None,
                 d: Optional[torch.Tensor] = None, id: Optional[torch.Tensor] = None):
        self.t = {k: tensors[k] for k in STATE_FIELDS}
        self.mat, self.d, self.id = mat, d, id

    @property
    def n(self) -> int:
        return int(self.t["x"].shape[0])

    def __getitem__(self, k):
        if k in ("mat", "d", "id"):
            return getattr(self, k)
        return self.t[k]

    @classmethod
    def empty(cls, n: int, device="cuda", with_mat=True, with_d=False, with_id=False):
        t = {k: torch.empty(n, dtype=torch.float64, device=device) for k in STATE_FIELDS}
        mat = torch.empty(n, dtype=torch.int32, device=device) if with_mat else None
        d = torch.empty(n, dtype=torch.float64, device=device) if with_d else None
        ids = torch.empty(n, dtype=torch.int64, device=device) if with_id else None
        return cls(t, mat, d, ids)

    def like(self) -> "State":
        return State.empty(self.n, self.t["x"].device, self.mat is not None, self.d is not None,
                           self.id is not None)

    @classmethod
    def from_numpy(cls, s: dict, device="cuda", with_id=True):
        t = {k: torch.as_tensor(s[k], dtype=torch.float64).to(device).contiguous()
             for k in STATE_FIELDS}
        mat = torch.as_tensor(s["mat"], dtype=torch.int32).to(device).contiguous()
        d = None
        if s.get("d") is not None:
            d = torch.as_tensor(s["d"], dtype=torch.float64).to(device).contiguous()
        ids = torch.arange(t["x"].shape[0], dtype=torch.int64, device=device) if with_id else None
        return cls(t, mat, d, ids)

    def numpy(self) -> dict:
        out = {k: v.cpu().numpy() for k, v in self.t.items()}
        if self.mat is not None:
            out["mat"] = self.mat.cpu().numpy()
        if self.d is not None:
            out["d"] = self.d.cpu().numpy()
        if self.id is not None:
            out["id"] = self.id.cpu().numpy()
        return out

    def c(self) -> N.CsphState:
        s = N.CsphState()
        s.n = self.n
        for k in STATE_FIELDS:
            setattr(s, k, _dp(self.t[k]))
        s.mat = _ip(self.mat)
        s.d = _dp(self.d)
        s.id = _lp(self.id)
        return s


class Workspace:
    """Caller-owned device scratch for the library (grown on demand)."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = torch.empty(1 << 20, dtype=torch.uint8, device=device)

    def ensure(self, nbytes: int):
        if self.buf.numel() < nbytes:
            self.buf = torch.empty(int(nbytes * 1.25) + (1 << 20), dtype=torch.uint8,
                                   device=self.device)

    @property
    def ptr(self):
        return C.c_void_p(self.buf.data_ptr())

    @property
    def nbytes(self):
        return int(self.buf.numel())


_default_ws: Dict[str, Workspace] = {}


def default_workspace(device="cuda") -> Workspace:
    key = str(torch.device(device))
    if key not in _default_ws:
        _default_ws[key] = Workspace(device)
    return _default_ws[key]


def _with_ws(fn, ws: Workspace, where: str, accept=()):
    """Call fn(ws_ptr, ws_bytes, needed_ptr); grow the workspace on CSPH_ECAPACITY (a call
    that bins twice, such as an RK2 step or its VJP, can learn its needs one mesh at a time).
    Statuses in ``accept`` are returned instead of raised."""
    needed = C.c_size_t(0)
    for _ in range(4):
        st = fn(ws.ptr, ws.nbytes, C.byref(needed))
        if st == N.CSPH_ECAPACITY and needed.value > ws.nbytes:
            ws.ensure(needed.value)
            continue
        if st in accept:
            return st
        N.check(st, where)
        return st
    N.check(st, where)
    return st


def profile_enable(on: bool = True):
    N.check(N.load().csph_profile_enable(1 if on else 0), "csph_profile_enable")


def profile_groups(groups=None):
    """Time only the named groups (names of PROF_GROUPS; None: all) while timing is on."""
    if groups is None:
        mask = 0xFFFFFFFF
    else:
        mask = 0
        for g in groups:
            mask |= 1 << N.PROF_GROUPS.index(g)
    N.check(N.load().csph_profile_groups(mask), "csph_profile_groups")


def profile_read() -> Dict[str, Tuple[int, float]]:
    """{group: (launches, total ms)} since the previous read (waits for the events)."""
    pr = N.CsphProfile()
    N.check(N.load().csph_profile_read(C.byref(pr)), "csph_profile_read")
    return {g: (int(pr.launches[k]), float(pr.ms[k])) for k, g in enumerate(N.PROF_GROUPS)}


def version() -> str:
    return N.load().csph_version().decode()


def workspace_size(n: int, ncell: int, params: Params) -> int:
    p = params.c()
    return int(N.load().csph_workspace_size(n, ncell, C.byref(p)))


def csph_grid_build(x, y, z, params: Params, d=None, ws: Optional[Workspace] = None,
                    stream=None) -> N.CsphGrid:
    L = N.load()
    ws = ws or default_workspace(x.device)
    g = N.CsphGrid()
    p = params.c()
    st = L.csph_grid_build(_dp(x), _dp(y), _dp(z), x.shape[0], C.byref(p), _dp(d), C.byref(g),
                           ws.ptr, ws.nbytes, _stream(stream))
    N.check(st, "csph_grid_build")
    return g


def csph_bin(x, y, z, grid: N.CsphGrid, ws: Optional[Workspace] = None, stream=None):
    """(key uint32-as-int64 view, perm int32, cell_start int32 [nkey + 1]) of sec. 4.2
    binning, keys as grid.key_mode (from the params of csph_grid_build) says."""
    L = N.load()
    ws = ws or default_workspace(x.device)
    n = x.shape[0]
    key = torch.empty(max(n, 1), dtype=torch.int32, device=x.device)
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=x.device)
    cs = torch.empty(grid.nkey + 1, dtype=torch.int32, device=x.device)
    _with_ws(lambda w, b, nd: L.csph_bin(_dp(x), _dp(y), _dp(z), n, C.byref(grid),
                                         C.cast(C.c_void_p(key.data_ptr()), C.POINTER(C.c_uint32)),
                                         _ip(perm), _ip(cs), cs.shape[0], w, b, nd,
                                         _stream(stream)), ws, "csph_bin")
    return key[:n].to(torch.int64) & 0xFFFFFFFF, perm[:n], cs


def csph_neighbors(state: State, params: Params, ws: Optional[Workspace] = None, stream=None):
    """CSR (offsets int64 [n+1], idx int32 [nnz]) of the FP64 neighbour sets."""
    L = N.load()
    ws = ws or default_workspace(state["x"].device)
    n = state.n
    off = torch.empty(n + 1, dtype=torch.int64, device=state["x"].device)
    s = state.c()
    p = params.c()
    nnz = C.c_int64(0)
    _with_ws(lambda w, b, nd: L.csph_neighbors(C.byref(s), C.byref(p), _lp(off), None, 0,
                                               C.byref(nnz), w, b, nd, _stream(stream)), ws,
             "csph_neighbors(count)")
    idx = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=state["x"].device)
    _with_ws(lambda w, b, nd: L.csph_neighbors(C.byref(s), C.byref(p), _lp(off), _ip(idx),
                                               idx.shape[0], C.byref(nnz), w, b, nd,
                                               _stream(stream)), ws, "csph_neighbors")
    return off, idx[:nnz.value]


def csph_rates(state: State, params: Params, t: float = 0.0, ws: Optional[Workspace] = None,
               stream=None, want_signal=True, want_count=True):
    """Rates (drho, dvx, dvy, dvz, dE) in the state's order, plus signal speed and |N(i)|.
    A non-physical state does not raise: out["nonphys"] counts the particles concerned and
    out["status"] is CSPH_ENONPHYS."""
    L = N.load()
    dev = state["x"].device
    ws = ws or default_workspace(dev)
    n = state.n
    out = {k: torch.empty(n, dtype=torch.float64, device=dev)
           for k in ("drho", "dvx", "dvy", "dvz", "dE")}
    sig = torch.empty(n, dtype=torch.float64, device=dev) if want_signal else None
    cnt = torch.empty(n, dtype=torch.int32, device=dev) if want_count else None
    nonphys = torch.zeros(1, dtype=torch.int64, device=dev)
    ro = N.CsphRatesOut(*[_dp(out[k]) for k in ("drho", "dvx", "dvy", "dvz", "dE")])
    s = state.c()
    p = params.c()
    status = _with_ws(lambda w, b, nd: L.csph_rates(C.byref(s), C.byref(p), float(t), ro,
                                                    _dp(sig), _ip(cnt), _lp(nonphys), w, b, nd,
                                                    _stream(stream)), ws, "csph_rates",
                      accept=(N.CSPH_ENONPHYS,))
    out["status"] = status
    if sig is not None:
        out["signal"] = sig
    if cnt is not None:
        out["nbr_count"] = cnt
    out["nonphys"] = nonphys
    return out


class StepScalars:
    """Device scalars a run of steps carries: time, last dt, totals, non-physical count."""

    def __init__(self, device="cuda", t0: float = 0.0):
        self.t = torch.full((1,), float(t0), dtype=torch.float64, device=device)
        self.dt = torch.zeros(1, dtype=torch.float64, device=device)
        self.totals = torch.zeros(10, dtype=torch.float64, device=device)
        self.nonphys = torch.zeros(1, dtype=torch.int64, device=device)


def csph_step(s_in: State, params: Params, sc: StepScalars, s_out: Optional[State] = None,
              dt_in: float = 0.0, nbr_count: Optional[torch.Tensor] = None,
              ws: Optional[Workspace] = None, stream=None, totals: bool = True) -> State:
    """One step s_in -> s_out (allocated when None); returns s_out.  With
    params.check_nonphys the call waits for its kernels and raises NonPhysicalState (the
    step is complete) if the EOS met a non-physical state."""
    L = N.load()
    ws = ws or default_workspace(s_in["x"].device)
    if s_out is None:
        s_out = s_in.like() if params.reorder else s_in
    a, b_ = s_in.c(), s_out.c()
    p = params.c()
    _with_ws(lambda w, nb, nd: L.csph_step(C.byref(a), C.byref(b_), C.byref(p), _dp(sc.t),
                                           float(dt_in), _dp(sc.dt),
                                           _dp(sc.totals) if totals else None, _ip(nbr_count),
                                           _lp(sc.nonphys), w, nb, nd, _stream(stream)), ws,
             "csph_step")
    return s_out


def csph_step_voronoi(s_in: State, params: Params, sc: StepScalars, sites: torch.Tensor,
                      owner: torch.Tensor, site_particles: torch.Tensor,
                      site_pairs: Optional[torch.Tensor] = None, s_out: Optional[State] = None,
                      dt_in: float = 0.0, nbr_count: Optional[torch.Tensor] = None,
                      ws: Optional[Workspace] = None, stream=None, totals: bool = True) -> State:
    """csph_step plus the Voronoi ownership of the new positions (owner int32 [n] in s_out's
    order, site_particles / site_pairs int64 [K]), computed inside the step's update."""
    L = N.load()
    ws = ws or default_workspace(s_in["x"].device)
    if s_out is None:
        s_out = s_in.like() if params.reorder else s_in
    if sites.dtype != torch.float64 or not sites.is_contiguous():
        sites = sites.to(torch.float64).contiguous()
    K = sites.shape[0]
    a, b_ = s_in.c(), s_out.c()
    p = params.c()
    _with_ws(lambda w, nb, nd: L.csph_step_voronoi(
        C.byref(a), C.byref(b_), C.byref(p), _dp(sc.t), float(dt_in), _dp(sc.dt),
        _dp(sc.totals) if totals else None, _ip(nbr_count), _lp(sc.nonphys), _dp(sites), K,
        _ip(owner), _lp(site_particles), _lp(site_pairs), w, nb, nd, _stream(stream)), ws,
        "csph_step_voronoi")
    return s_out


def csph_step_static(s_in: State, params: Params, sc: StepScalars, s_out: State,
                     dt_in: float = 0.0, nbr_count: Optional[torch.Tensor] = None,
                     stream=None, totals: bool = True) -> State:
    """csph_step with the library's own static scratch instead of a caller workspace: the
    library call allocates nothing (for callers that cannot allocate).  s_out must be given;
    it may be s_in itself when params.reorder is False."""
    L = N.load()
    a, b_ = s_in.c(), s_out.c()
    p = params.c()
    st = L.csph_step_static(C.byref(a), C.byref(b_), C.byref(p), _dp(sc.t), float(dt_in),
                            _dp(sc.dt), _dp(sc.totals) if totals else None, _ip(nbr_count),
                            _lp(sc.nonphys), _stream(stream))
    N.check(st, "csph_step_static")
    return s_out


def domain_mesh(lo, hi, params: Params, device="cuda", ws: Optional[Workspace] = None,
                stream=None) -> N.CsphGrid:
    """The mesh csph_grid_build makes for the box [lo, hi] (its two corners as the points), for
    csph_step_mesh: cells of params.cell_size (or the support), covering the box."""
    pts = torch.tensor([lo, hi], dtype=torch.float64, device=device)
    return csph_grid_build(pts[:, 0].contiguous(), pts[:, 1].contiguous(),
                           pts[:, 2].contiguous(), params, ws=ws, stream=stream)


def csph_step_mesh(s_in: State, params: Params, sc: StepScalars, mesh: N.CsphGrid,
                   s_out: Optional[State] = None, dt_in: float = 0.0,
                   nbr_count: Optional[torch.Tensor] = None,
                   outside: Optional[torch.Tensor] = None, ws: Optional[Workspace] = None,
                   stream=None, totals: bool = True) -> State:
    """csph_step on the caller's mesh (e.g. domain_mesh): no host synchronisation, so a
    sequence of these calls can be captured in a graph (size ``ws`` with an eager call first).
    ``outside`` (int64 [1], device, accumulated) counts the particles off the mesh."""
    L = N.load()
    ws = ws or default_workspace(s_in["x"].device)
    if s_out is None:
        s_out = s_in.like() if params.reorder else s_in
    a, b_ = s_in.c(), s_out.c()
    p = params.c()
    _with_ws(lambda w, nb, nd: L.csph_step_mesh(C.byref(a), C.byref(b_), C.byref(p),
                                                C.byref(mesh), _dp(sc.t), float(dt_in),
                                                _dp(sc.dt), _dp(sc.totals) if totals else None,
                                                _ip(nbr_count), _lp(sc.nonphys), _lp(outside), w,
                                                nb, nd, _stream(stream)), ws, "csph_step_mesh")
    return s_out


def voronoi_assign(x, y, z, sites: torch.Tensor, nbr_count: Optional[torch.Tensor] = None,
                   owner: Optional[torch.Tensor] = None, stream=None,
                   site_particles: Optional[torch.Tensor] = None,
                   site_pairs: Optional[torch.Tensor] = None):
    """(owner int32 [n], site_particles int64 [K], site_pairs int64 [K] or None).

    Output buffers may be passed in (owner int32 [>= n], site_particles and
    site_pairs int64 [K]); site_pairs is only written when nbr_count is given.
    """
    L = N.load()
    n = x.shape[0]
    K = sites.shape[0]
    if sites.dtype != torch.float64 or not sites.is_contiguous():
        sites = sites.to(torch.float64).contiguous()
    if owner is None:
        owner = torch.empty(max(n, 1), dtype=torch.int32, device=x.device)
    sp = site_particles
    if sp is None:
        sp = torch.empty(K, dtype=torch.int64, device=x.device)
    spairs = None
    if nbr_count is not None:
        spairs = site_pairs
        if spairs is None:
            spairs = torch.empty(K, dtype=torch.int64, device=x.device)
    for name, buf, dt, need in (("owner", owner, torch.int32, n), ("site_particles", sp, torch.int64, K),
                                ("site_pairs", spairs, torch.int64, K)):
        if buf is not None and (buf.dtype != dt or buf.numel() < need or not buf.is_contiguous()):
            raise ValueError(f"voronoi_assign: {name} must be contiguous {dt} with >= {need} entries")
    st = L.voronoi_assign(_dp(x), _dp(y), _dp(z), n, _dp(sites), K, _ip(nbr_count), _ip(owner),
                          _lp(sp), _lp(spairs), _stream(stream))
    N.check(st, "voronoi_assign")
    return owner[:n], sp, spairs


def csph_init_energy(rho, pres, vx, vy, vz, mat, params: Params, stream=None):
    L = N.load()
    n = rho.shape[0]
    E = torch.empty(n, dtype=torch.float64, device=rho.device)
    p = params.c()
    st = L.csph_init_energy(_dp(rho), _dp(pres), _dp(vx), _dp(vy), _dp(vz), _ip(mat), n,
                            C.byref(p), _dp(E), _stream(stream))
    N.check(st, "csph_init_energy")
    return E


GRAD_FIELDS = ("x", "y", "z", "vx", "vy", "vz", "rho", "E")


def _grad_struct(g: Dict[str, torch.Tensor]) -> N.CsphGrad:
    return N.CsphGrad(*[_dp(g[k]) for k in GRAD_FIELDS])


def zeros_grad(n: int, device="cuda") -> Dict[str, torch.Tensor]:
    return {k: torch.zeros(n, dtype=torch.float64, device=device) for k in GRAD_FIELDS}


def csph_rates_vjp(state: State, params: Params, cot: Dict[str, torch.Tensor],
                   g_state: Optional[Dict[str, torch.Tensor]] = None,
                   g_eos: Optional[torch.Tensor] = None, ws: Optional[Workspace] = None,
                   stream=None, t: float = 0.0):
    """g_state += (d rates/d state)^T cot, g_eos += EOS-parameter part; returns both.
    ``t``: the time of the rates (the piston's position)."""
    L = N.load()
    dev = state["x"].device
    ws = ws or default_workspace(dev)
    if g_state is None:
        g_state = zeros_grad(state.n, dev)
    if g_eos is None:
        g_eos = torch.zeros(2 * len(params.eos), dtype=torch.float64, device=dev)
    a = N.CsphRatesOut(*[_dp(cot[k]) for k in ("drho", "dvx", "dvy", "dvz", "dE")])
    s = state.c()
    p = params.c()
    gs = _grad_struct(g_state)
    _with_ws(lambda w, b, nd: L.csph_rates_vjp(C.byref(s), C.byref(p), float(t), a, gs,
                                               _dp(g_eos), w, b, nd, _stream(stream)), ws,
             "csph_rates_vjp")
    return g_state, g_eos


def csph_step_vjp(s_n: State, params: Params, dt: float, g_next: Dict[str, torch.Tensor],
                  g_prev: Optional[Dict[str, torch.Tensor]] = None,
                  g_eos: Optional[torch.Tensor] = None, ws: Optional[Workspace] = None,
                  stream=None, t: float = 0.0):
    """Cotangent of s_n from that of the state after one step taken at time ``t`` with frozen
    dt."""
    L = N.load()
    dev = s_n["x"].device
    ws = ws or default_workspace(dev)
    if g_prev is None:
        g_prev = g_next
    if g_eos is None:
        g_eos = torch.zeros(2 * len(params.eos), dtype=torch.float64, device=dev)
    s = s_n.c()
    p = params.c()
    gn, gp = _grad_struct(g_next), _grad_struct(g_prev)
    _with_ws(lambda w, b, nd: L.csph_step_vjp(C.byref(s), C.byref(p), float(t), float(dt), gn,
                                              gp, _dp(g_eos), w, b, nd, _stream(stream)), ws,
             "csph_step_vjp")
    return g_prev, g_eos


def csph_step_vjp_cfl(s_n: State, params: Params, g_next: Dict[str, torch.Tensor],
                      g_prev: Optional[Dict[str, torch.Tensor]] = None,
                      g_eos: Optional[torch.Tensor] = None, ws: Optional[Workspace] = None,
                      stream=None, t: float = 0.0):
    """Cotangent of s_n from that of the state after one step taken at time ``t`` with the CFL
    time step (params.cfl > 0), the step's dependence through dt included; returns
    (g_prev, g_eos, dt), dt the step recomputed in FP64."""
    L = N.load()
    dev = s_n["x"].device
    ws = ws or default_workspace(dev)
    if g_prev is None:
        g_prev = g_next
    if g_eos is None:
        g_eos = torch.zeros(2 * len(params.eos), dtype=torch.float64, device=dev)
    s = s_n.c()
    p = params.c()
    gn, gp = _grad_struct(g_next), _grad_struct(g_prev)
    dt = C.c_double(0.0)
    _with_ws(lambda w, b, nd: L.csph_step_vjp_cfl(C.byref(s), C.byref(p), float(t), gn, gp,
                                                  _dp(g_eos), C.byref(dt), w, b, nd,
                                                  _stream(stream)), ws, "csph_step_vjp_cfl")
    return g_prev, g_eos, dt.value


def csph_init_energy_vjp(rho, pres, vx, vy, vz, mat, params: Params, gE, g_v=None, g_rho=None,
                         g_eos=None, ws: Optional[Workspace] = None, stream=None):
    L = N.load()
    ws = ws or default_workspace(rho.device)
    n = rho.shape[0]
    p = params.c()
    gv = g_v or (None, None, None)
    _with_ws(lambda w, b, nd: L.csph_init_energy_vjp(_dp(rho), _dp(pres), _dp(vx), _dp(vy),
                                                     _dp(vz), _ip(mat), n, C.byref(p), _dp(gE),
                                                     _dp(gv[0]), _dp(gv[1]), _dp(gv[2]),
                                                     _dp(g_rho), _dp(g_eos), w, b, nd,
                                                     _stream(stream)), ws,
             "csph_init_energy_vjp")


def state_from_workload(w, params: Params, device="cuda", with_id=True) -> State:
    """Device state of a synthetic workload: E built on the GPU from (rho, p, v)."""
    t = {k: torch.as_tensor(getattr(w, k), dtype=torch.float64).to(device).contiguous()
         for k in ("x", "y", "z", "vx", "vy", "vz", "rho", "m")}
    mat = torch.as_tensor(w.mat, dtype=torch.int32).to(device).contiguous()
    p = torch.as_tensor(w.p, dtype=torch.float64).to(device).contiguous()
    t["E"] = csph_init_energy(t["rho"], p, t["vx"], t["vy"], t["vz"], mat, params)
    ids = torch.arange(t["x"].shape[0], dtype=torch.int64, device=device) if with_id else None
    return State(t, mat, None, ids)


# ------------------------------------------------------------------ Voronoi balancer

@dataclass
class BalanceParams:
    """Weights of the generator move (eqs. BalancingOffsetPlusRot and TotalOffset)."""
    sigma: float = 0.5    # three-body weight
    theta: float = 0.25   # material-motion weight
    gamma: float = 1.0    # balancing-displacement scale
    dsh: float = 3.0      # D^sh, exchange-layer half width
    load: str = "pairs"   # "pairs" (site_pairs) or "particles" (site_particles)

    def c(self) -> N.CsphBalanceParams:
        return N.CsphBalanceParams(float(self.sigma), float(self.theta), float(self.gamma),
                                   float(self.dsh))


def _u32p(t):
    if t is not None:
        assert t.dtype == torch.int32 and t.is_contiguous() and t.is_cuda
    return _ptr(t, C.c_uint32)


def adjacency_matrix(bits: torch.Tensor, K: int) -> torch.Tensor:
    """Unpack the K x ceil(K/32) word bit matrix into a bool [K, K] tensor (host copy)."""
    w = bits.view(K, -1).cpu().to(torch.int64) & 0xFFFFFFFF
    cols = torch.arange(K)
    return ((w[:, cols // 32] >> (cols % 32)) & 1).bool()


def csph_balance_stats(x, y, z, owner, sites: torch.Tensor, dsh: float,
                       nbr_count: Optional[torch.Tensor] = None, ws: Optional[Workspace] = None,
                       stream=None) -> Dict[str, torch.Tensor]:
    """Loads, centres and the touching-subdomain bit matrix of the assignment ``owner``.

    Returns dict(particles int64 [K], pairs int64 [K] or None, centre float64 [K, 3],
    adjacency int32 [K, ceil(K/32)] (uint32 bit words)).
    """
    L = N.load()
    ws = ws or default_workspace(x.device)
    sites = sites.to(torch.float64).contiguous()
    K = sites.shape[0]
    n = x.shape[0]
    dev = x.device
    out = dict(particles=torch.empty(K, dtype=torch.int64, device=dev),
               pairs=torch.empty(K, dtype=torch.int64, device=dev) if nbr_count is not None else None,
               centre=torch.empty(K, 3, dtype=torch.float64, device=dev),
               adjacency=torch.empty(K, (K + 31) // 32, dtype=torch.int32, device=dev))
    _with_ws(lambda p, b, nd: L.csph_balance_stats(
        _dp(x), _dp(y), _dp(z), n, _ip(owner), _ip(nbr_count), _dp(sites), K, float(dsh),
        _lp(out["particles"]), _lp(out["pairs"]), _dp(out["centre"]), _u32p(out["adjacency"]),
        p, b, nd, _stream(stream)), ws, "csph_balance_stats")
    return out


def csph_balance_move(sites: torch.Tensor, stats: Dict[str, torch.Tensor], bp: BalanceParams,
                      stream=None):
    """One generator move from ``csph_balance_stats`` output: (new sites [K, 3], move_sum [1])."""
    L = N.load()
    sites = sites.to(torch.float64).contiguous()
    K = sites.shape[0]
    loads = stats["pairs"] if (bp.load == "pairs" and stats.get("pairs") is not None) \
        else stats["particles"]
    new = torch.empty_like(sites)
    ms = torch.empty(1, dtype=torch.float64, device=sites.device)
    p = bp.c()
    st = L.csph_balance_move(_dp(sites), K, _lp(loads.contiguous()), _dp(stats["centre"]),
                             _u32p(stats["adjacency"]), C.byref(p), _dp(new), _dp(ms),
                             _stream(stream))
    N.check(st, "csph_balance_move")
    return new, ms


# ------------------------------------------------------------------ Verlet lists

VLIST_CTL_BYTES = 48  # csph_vlist_ctl


def vlist_ctl(device="cuda") -> torch.Tensor:
    """Device storage for a csph_vlist_ctl (6 x 8 bytes)."""
    return torch.zeros(VLIST_CTL_BYTES // 8, dtype=torch.int64, device=device)


def vlist_ctl_read(ctl: torch.Tensor) -> Dict[str, float]:
    """Host copy of a csph_vlist_ctl (synchronises)."""
    import numpy as np
    raw = ctl.cpu().numpy().view(np.uint8)
    f = raw[:32].view(np.float64)
    return {"t_build": float(f[0]), "disp": float(f[1]), "margin": float(f[2]),
            "vw2": float(f[3]), "pairs": int(raw[32:40].view(np.int64)[0]),
            "steps": int(raw[40:44].view(np.int32)[0]), "valid": int(raw[44:48].view(np.int32)[0])}


def csph_vlist_build(s_in: State, s_out: State, params: Params, sc: StepScalars, beta: float,
                     cap: int, count: torch.Tensor, idx: torch.Tensor, x_ref: torch.Tensor,
                     ctl: Optional[torch.Tensor] = None, ws: Optional[Workspace] = None,
                     stream=None) -> int:
    """Renumber s_in into cell order in s_out and build the horizon lists; returns 0, or the
    longest list when it exceeds ``cap`` (the lists are then truncated).  ``ctl`` (from
    vlist_ctl) is reset for these lists."""
    L = N.load()
    ws = ws or default_workspace(s_in["x"].device)
    a, b_ = s_in.c(), s_out.c()
    p = params.c()
    mx = C.c_int32(0)
    needed = C.c_size_t(0)
    cp = C.c_void_p(ctl.data_ptr()) if ctl is not None else None
    for _ in range(3):
        st = L.csph_vlist_build(C.byref(a), C.byref(b_), C.byref(p), _dp(sc.t), float(beta),
                                int(cap), _ip(count), _ip(idx), _dp(x_ref), cp, C.byref(mx),
                                ws.ptr, ws.nbytes, C.byref(needed), _stream(stream))
        if st == N.CSPH_ECAPACITY and mx.value == 0 and needed.value > ws.nbytes:
            ws.ensure(needed.value)
            continue
        if st == N.CSPH_ECAPACITY and mx.value > 0:
            return int(mx.value)
        N.check(st, "csph_vlist_build")
        return 0
    N.check(st, "csph_vlist_build")
    return 0


def csph_step_vlist(s: State, params: Params, sc: StepScalars, count, idx, cap: int, x_ref,
                    ctl: torch.Tensor, dt_in: float = 0.0,
                    nbr_count: Optional[torch.Tensor] = None, ws: Optional[Workspace] = None,
                    stream=None, totals: bool = True) -> State:
    """One step in place from Verlet lists (s in the lists' order); a no-op once the device
    guard has found the lists stale (see csph_vlist_ctl)."""
    L = N.load()
    ws = ws or default_workspace(s["x"].device)
    a = s.c()
    p = params.c()
    cp = C.c_void_p(ctl.data_ptr())
    _with_ws(lambda w, nb, nd: L.csph_step_vlist(
        C.byref(a), C.byref(p), _dp(sc.t), float(dt_in), _dp(sc.dt),
        _dp(sc.totals) if totals else None, _ip(nbr_count), _lp(sc.nonphys), _ip(count),
        _ip(idx), int(cap), _dp(x_ref), cp, w, nb, nd, _stream(stream)), ws,
        "csph_step_vlist")
    return s


class VerletRun:
    """Steps from Verlet lists (sec. 4.2): lists of the partners within (1 + beta) H are
    rebuilt every ``n_upd`` steps, and earlier when the displacement bound
    2 max|r - r_ref| + 2 |v_wall| (t - t_build) reaches beta H, so that every step
    evaluates exactly N(i).  The bound is checked by each list step on the device: the
    driver issues up to ``n_upd`` steps without waiting, then reads the lists' control
    block once (one synchronisation per batch), and rebuilds and re-issues what a stale
    list skipped.  The state is renumbered into cell order at each rebuild.  ``cap`` is the
    list capacity per particle (grown on overflow)."""

    def __init__(self, state: State, params: Params, beta: float = 0.3, n_upd: int = 10,
                 cap: Optional[int] = None, ws: Optional[Workspace] = None):
        if params.h_mode != "fixed":
            raise ValueError("Verlet lists need fixed-h mode")
        self.params, self.beta, self.n_upd = params, float(beta), int(n_upd)
        self.ws = ws or default_workspace(state["x"].device)
        n = state.n
        dev = state["x"].device
        H = params.kappa * params.h
        # partners within (1 + beta) H on a unit-density lattice, with room for compression
        cap = int(cap) if cap else int(4.5 * ((1.0 + self.beta) * H) ** 3) + 32
        self.cap = -(-cap // 8) * 8  # whole 8-entry chunks
        self.state, self.other = state, state.like()
        self.count = torch.zeros(max(n, 1), dtype=torch.int32, device=dev)
        self.idx = torch.empty(max(n, 1) * self.cap, dtype=torch.int32, device=dev)
        self.x_ref = torch.empty(3 * max(n, 1), dtype=torch.float64, device=dev)
        self.ctl = vlist_ctl(dev)
        self.since = None   # list steps taken since the build (None: no lists yet)
        self.valid = False
        self.builds = 0
        self.pairs = 0      # directed pairs evaluated by list steps (read at synchronisations)
        self.H = H

    def _build(self, sc: StepScalars):
        while True:
            over = csph_vlist_build(self.state, self.other, self.params, sc, self.beta, self.cap,
                                    self.count, self.idx, self.x_ref, self.ctl, ws=self.ws)
            if over == 0:
                break
            self.cap = -(-(int(over * 1.25) + 8) // 8) * 8
            self.idx = torch.empty(max(self.state.n, 1) * self.cap, dtype=torch.int32,
                                   device=self.idx.device)
        self.state, self.other = self.other, self.state
        self.since = 0
        self.valid = True
        self._pairs_seen = 0  # the control block's pair count restarts at a build
        self.builds += 1

    def advance(self, sc: StepScalars, k: int, nbr_count: Optional[torch.Tensor] = None,
                dt_in: float = 0.0, totals: bool = True) -> State:
        """k exact steps; one synchronisation per batch of up to n_upd list steps."""
        done = 0
        while done < k:
            if self.since is None or self.since >= self.n_upd or not self.valid:
                self._build(sc)
            m = min(k - done, self.n_upd - self.since)
            for _ in range(m):
                csph_step_vlist(self.state, self.params, sc, self.count, self.idx, self.cap,
                                self.x_ref, self.ctl, dt_in=dt_in, nbr_count=nbr_count,
                                ws=self.ws, totals=totals)
            c = vlist_ctl_read(self.ctl)
            taken = c["steps"] - self.since
            self.pairs += c["pairs"] - self._pairs_seen
            self._pairs_seen = c["pairs"]
            self.since = c["steps"]
            self.valid = bool(c["valid"])
            done += taken
        return self.state

    def step(self, sc: StepScalars, nbr_count: Optional[torch.Tensor] = None,
             dt_in: float = 0.0, totals: bool = True) -> State:
        return self.advance(sc, 1, nbr_count=nbr_count, dt_in=dt_in, totals=totals)
