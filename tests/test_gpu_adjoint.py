"""GPU adjoint: csph_rates_vjp, csph_step_vjp, csph_init_energy_vjp and the
checkpointed rollout against the FP64 CPU reference gradient (autograd of
oracle/torch_ref.py) and against central finite differences."""
import numpy as np
import pytest
import torch

import csph_inputs as ci
import oracle as O
import paper_1805_05128_amd as P
from oracle import torch_ref as T

pytestmark = pytest.mark.gpu
DEV = "cuda"
F8 = T.FIELDS8


def system(n=8, seed=3, two_mat=True):
    w = ci.jittered_block(n, n, n, seed=seed, amp=0.05)
    rng = np.random.default_rng(seed)
    w.vx = rng.uniform(-0.3, 0.3, w.n)
    w.vy = rng.uniform(-0.3, 0.3, w.n)
    w.vz = rng.uniform(-0.3, 0.3, w.n)
    w.rho = rng.uniform(0.8, 1.3, w.n)
    w.p = rng.uniform(0.5, 1.5, w.n)
    w.m = w.rho.copy()
    if two_mat:
        w.mat = (w.x > n / 2).astype(np.int32)
        w.eos = [(0, 1.4, 0.0), (1, 3.0, 0.4)]
    return w


def tparams(w, grad=False):
    g = torch.tensor([e[1] for e in w.eos], dtype=torch.float64, requires_grad=grad)
    pi = torch.tensor([e[2] for e in w.eos], dtype=torch.float64, requires_grad=grad)
    return [e[0] for e in w.eos], g, pi


def relmax(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def slab_system(seed=8):
    """5 x 24 x 5 block on unit cells (24 cell rows): the internal y-slab cell order
    has a full 16-row slab and a short one."""
    w = ci.jittered_block(5, 24, 5, seed=seed, amp=0.05)
    rng = np.random.default_rng(seed)
    w.vx = rng.uniform(-0.3, 0.3, w.n)
    w.vy = rng.uniform(-0.3, 0.3, w.n)
    w.vz = rng.uniform(-0.3, 0.3, w.n)
    w.rho = rng.uniform(0.8, 1.3, w.n)
    w.p = rng.uniform(0.5, 1.5, w.n)
    w.m = w.rho.copy()
    w.mat = (w.y > 12).astype(np.int32)
    w.eos = [(0, 1.4, 0.0), (1, 3.0, 0.4)]
    w.cell_size = 1.0
    return w


@pytest.mark.parametrize("make", [system, slab_system], ids=["block", "slab"])
def test_rates_vjp_matches_autograd(make):
    w = make()
    params = P.Params.from_workload(w)
    g = P.state_from_workload(w, params, DEV)
    s = {k: g[k].cpu().numpy() for k in F8}
    s["m"] = w.m
    s["mat"] = w.mat
    rng = np.random.default_rng(1)
    cot = {k: rng.standard_normal(w.n) for k in ("drho", "dvx", "dvy", "dvz", "dE")}
    gs, ge = P.csph_rates_vjp(g, params, {k: torch.as_tensor(v, device=DEV) for k, v in cot.items()})
    et, gg, pi = tparams(w, True)
    st = {k: torch.as_tensor(s[k]).clone().requires_grad_(True) for k in F8}
    cfg = O.cfg_for(w)
    out = T.rates_torch(st, torch.as_tensor(w.m), torch.as_tensor(w.mat).long(), et, gg, pi,
                        T.pairs_of(cfg, s), w.kappa * w.h)
    J = sum((o * torch.as_tensor(cot[k])).sum()
            for o, k in zip(out, ("drho", "dvx", "dvy", "dvz", "dE")))
    ref = torch.autograd.grad(J, [st[k] for k in F8] + [gg, pi])
    for a, k in enumerate(F8):
        e = relmax(gs[k].cpu().numpy(), ref[a].numpy())
        assert e <= 1e-10, (k, e)
    ge = ge.cpu().numpy()
    assert relmax(ge[0::2], ref[8].numpy()) <= 1e-10
    assert abs(ge[3] - float(ref[9][1])) <= 1e-10 * abs(float(ref[9][1]))


def test_step_vjp_matches_autograd_and_dot_product():
    w = system(seed=5)
    params = P.Params.from_workload(w, reorder=False)
    g = P.state_from_workload(w, params, DEV)
    s = {k: g[k].cpu().numpy() for k in F8}
    s["m"] = w.m
    s["mat"] = w.mat
    dt = 0.04
    rng = np.random.default_rng(2)
    lam = {k: rng.standard_normal(w.n) for k in F8}
    gn = {k: torch.as_tensor(v, device=DEV).clone() for k, v in lam.items()}
    gp, ge = P.csph_step_vjp(g, params, dt, gn, g_prev={k: torch.empty_like(v) for k, v in gn.items()})
    et, gg, pi = tparams(w, True)
    st = {k: torch.as_tensor(s[k]).clone().requires_grad_(True) for k in F8}
    out = T.step_torch(st, torch.as_tensor(w.m), torch.as_tensor(w.mat).long(), et, gg, pi,
                       T.pairs_of(O.cfg_for(w), s), w.kappa * w.h, dt)
    J = sum((out[k] * torch.as_tensor(lam[k])).sum() for k in F8)
    ref = torch.autograd.grad(J, [st[k] for k in F8] + [gg, pi])
    for a, k in enumerate(F8):
        assert relmax(gp[k].cpu().numpy(), ref[a].numpy()) <= 1e-10, k
    # dot-product test against the GPU forward step: <lam, J d> = <J^T lam, d>
    d = {k: rng.standard_normal(w.n) for k in F8}
    eps = 1e-6
    replay = P.Params.from_workload(w, reorder=False, cfl=0.0)

    def fwd(sign):
        t = {k: g[k] + sign * eps * torch.as_tensor(d[k], device=DEV) for k in F8}
        t["m"] = g["m"]
        st2 = P.State(t, g.mat)
        P.csph_step(st2, replay, P.StepScalars(DEV), s_out=st2, dt_in=dt)
        return {k: st2[k].cpu().numpy() for k in F8}

    fp, fm = fwd(1), fwd(-1)
    jvp = sum(float(((fp[k] - fm[k]) / (2 * eps) * lam[k]).sum()) for k in F8)
    vjp = sum(float((gp[k].cpu().numpy() * d[k]).sum()) for k in F8)
    assert abs(jvp - vjp) <= 1e-7 * max(abs(vjp), 1.0), (jvp, vjp)


def test_init_energy_vjp_matches_autograd():
    w = system()
    params = P.Params.from_workload(w)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64), device=DEV)
    gE = np.random.default_rng(4).standard_normal(w.n)
    gv = [torch.zeros(w.n, dtype=torch.float64, device=DEV) for _ in range(3)]
    grho = torch.zeros(w.n, dtype=torch.float64, device=DEV)
    geos = torch.zeros(4, dtype=torch.float64, device=DEV)
    P.csph_init_energy_vjp(t(w.rho), t(w.p), t(w.vx), t(w.vy), t(w.vz),
                           torch.as_tensor(w.mat, device=DEV), params, t(gE), g_v=gv, g_rho=grho,
                           g_eos=geos)
    et, gg, pi = tparams(w, True)
    vx = torch.as_tensor(w.vx).clone().requires_grad_(True)
    rho = torch.as_tensor(w.rho).clone().requires_grad_(True)
    E = T.init_energy_torch(rho, torch.as_tensor(w.p), vx, torch.as_tensor(w.vy),
                            torch.as_tensor(w.vz), torch.as_tensor(w.mat).long(), et, gg, pi)
    ref = torch.autograd.grad((E * torch.as_tensor(gE)).sum(), [vx, rho, gg, pi])
    assert relmax(gv[0].cpu().numpy(), ref[0].numpy()) <= 1e-13
    assert relmax(grho.cpu().numpy(), ref[1].numpy()) <= 1e-13
    assert relmax(geos.cpu().numpy()[0::2], ref[2].numpy()) <= 1e-12
    assert abs(geos.cpu().numpy()[3] - float(ref[3][1])) <= 1e-12 * abs(float(ref[3][1]))


def _base(w, params):
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64), device=DEV).contiguous()
    return dict(x=t(w.x), y=t(w.y), z=t(w.z), rho=t(w.rho), p=t(w.p), m=t(w.m),
                mat=torch.as_tensor(w.mat, dtype=torch.int32, device=DEV))


def _objective(out, mask, m):
    return (out["vx"][mask] * m[mask]).sum()


def test_rollout_gradient_matches_reference_and_fd():
    w = system(n=8, seed=7)
    params = P.Params.from_workload(w, cfl=0.3)
    base = _base(w, params)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64), device=DEV)
    v0 = [t(w.vx).requires_grad_(True), t(w.vy).requires_grad_(True), t(w.vz).requires_grad_(True)]
    gamma = torch.tensor([e[1] for e in w.eos], dtype=torch.float64, device=DEV,
                         requires_grad=True)
    nsteps, every = 12, 5
    # the dt sequence of the oracle's run (CFL rule), replayed by both sides
    cfg = O.cfg_for(w)
    so, to, dts = O.state_from(w, cfg), 0.0, []
    for _ in range(nsteps):
        so, to, dt, _ = O.step(cfg, so, t=to)
        dts.append(dt)
    info = {}
    out = P.rollout(*v0, gamma, base, params, nsteps, every, info=info)
    # the GPU's own CFL steps agree with the oracle's
    assert np.allclose(info["dts"], dts, rtol=1e-13, atol=0.0)
    out = P.rollout(*v0, gamma, base, params, nsteps, every, dts=dts)
    mask = out["x"].detach() > 4.0
    J = _objective(out, mask, base["m"])
    grads = torch.autograd.grad(J, v0 + [gamma])
    assert len(dts) == nsteps and all(d > 0 for d in dts)
    # FP64 CPU reference: torch autograd over the same dt sequence
    et, gg, pi = tparams(w, True)
    gg = gg.clone().detach().requires_grad_(True)
    mat = torch.as_tensor(w.mat).long()
    m = torch.as_tensor(w.m)
    vr = [torch.as_tensor(a).clone().requires_grad_(True) for a in (w.vx, w.vy, w.vz)]
    E0 = T.init_energy_torch(torch.as_tensor(w.rho), torch.as_tensor(w.p), *vr, mat, et, gg, pi)
    st = {"x": torch.as_tensor(w.x), "y": torch.as_tensor(w.y), "z": torch.as_tensor(w.z),
          "vx": vr[0], "vy": vr[1], "vz": vr[2], "rho": torch.as_tensor(w.rho), "E": E0}
    for k in range(nsteps):
        pairs = T.pairs_of(cfg, {kk: st[kk].detach().numpy() for kk in ("x", "y", "z")})
        st = T.step_torch(st, m, mat, et, gg, pi, pairs, w.kappa * w.h, dts[k])
    mref = st["x"].detach() > 4.0
    assert torch.equal(mref, mask.cpu())
    Jr = (st["vx"][mref] * m[mref]).sum()
    ref = torch.autograd.grad(Jr, vr + [gg])
    assert abs(float(J.detach()) - float(Jr.detach())) <= 1e-11 * abs(float(Jr.detach()))
    for a in range(3):
        assert relmax(grads[a].cpu().numpy(), ref[a].numpy()) <= 1e-9, a
    assert relmax(grads[3].cpu().numpy(), ref[3].numpy()) <= 1e-9
    # central finite differences of the GPU forward with the dt sequence replayed
    rng = np.random.default_rng(11)
    for trial in range(4):
        d = [rng.standard_normal(w.n) for _ in range(3)]
        dg = rng.standard_normal(2)
        eps = 1e-6

        def Jat(sign):
            vv = [v0[a].detach() + sign * eps * t(d[a]) for a in range(3)]
            gm = gamma.detach() + sign * eps * t(dg)
            o = P.rollout(*vv, gm, base, params, nsteps, every, dts=dts)
            return float(_objective(o, mask, base["m"]))

        fd = (Jat(1) - Jat(-1)) / (2 * eps)
        pred = sum(float((grads[a].cpu().numpy() * d[a]).sum()) for a in range(3)) + \
            float((grads[3].cpu().numpy() * dg).sum())
        assert abs(fd - pred) <= 1e-4 * max(abs(pred), 1e-8), (trial, fd, pred)


def test_window_rollout_from_a_mid_run_state():
    """A rollout that starts from a state of a longer run (x, v, rho, E; E held fixed):
    gradients w.r.t. the window's velocities and gamma against the FP64 CPU reference
    (autograd over the same dt sequence) and central differences."""
    w = system(n=8, seed=12)
    cfg = O.cfg_for(w)
    s = O.state_from(w, cfg)
    t0 = 0.0
    for _ in range(4):  # the run before the window, on the oracle
        s, t0, _, _ = O.step(cfg, s, t=t0)
    params = P.Params.from_workload(w, cfl=0.3)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64), device=DEV).contiguous()
    base = dict(x=t(s["x"]), y=t(s["y"]), z=t(s["z"]), rho=t(s["rho"]), E=t(s["E"]),
                m=t(s["m"]), mat=torch.as_tensor(s["mat"], dtype=torch.int32, device=DEV))
    v0 = [t(s[k]).requires_grad_(True) for k in ("vx", "vy", "vz")]
    gamma = torch.tensor([e[1] for e in w.eos], dtype=torch.float64, device=DEV,
                         requires_grad=True)
    nsteps, every = 5, 5  # one checkpoint, the other states recomputed
    so, to, dts = s, t0, []
    for _ in range(nsteps):  # the oracle's dt sequence for the window, replayed by both sides
        so, to, dt, _ = O.step(cfg, so, t=to)
        dts.append(dt)
    out = P.rollout(*v0, gamma, base, params, nsteps, every, dts=dts)
    mask = out["z"].detach() > 4.0
    J = (out["vz"][mask] * base["m"][mask]).sum()
    grads = torch.autograd.grad(J, v0 + [gamma])
    et, gg, pi = tparams(w, True)
    gg = gg.clone().detach().requires_grad_(True)
    mat = torch.as_tensor(s["mat"]).long()
    m = torch.as_tensor(s["m"])
    vr = [torch.as_tensor(s[k]).clone().requires_grad_(True) for k in ("vx", "vy", "vz")]
    st = {"x": torch.as_tensor(s["x"]), "y": torch.as_tensor(s["y"]),
          "z": torch.as_tensor(s["z"]), "vx": vr[0], "vy": vr[1], "vz": vr[2],
          "rho": torch.as_tensor(s["rho"]), "E": torch.as_tensor(s["E"])}
    for k in range(nsteps):
        pairs = T.pairs_of(cfg, {kk: st[kk].detach().numpy() for kk in ("x", "y", "z")})
        st = T.step_torch(st, m, mat, et, gg, pi, pairs, w.kappa * w.h, dts[k])
    mref = st["z"].detach() > 4.0
    assert torch.equal(mref, mask.cpu())
    Jr = (st["vz"][mref] * m[mref]).sum()
    ref = torch.autograd.grad(Jr, vr + [gg])
    assert abs(float(J.detach()) - float(Jr.detach())) <= 1e-11 * abs(float(Jr.detach()))
    for a in range(3):
        assert relmax(grads[a].cpu().numpy(), ref[a].numpy()) <= 1e-9, a
    assert relmax(grads[3].cpu().numpy(), ref[3].numpy()) <= 1e-9
    # E is held fixed: the gradient of the final state does not pass through an E0(v0) map
    rng = np.random.default_rng(5)
    for trial in range(3):
        d = [rng.standard_normal(w.n) for _ in range(3)]
        eps = 1e-6

        def vz_at(sign):
            vv = [v0[a].detach() + sign * eps * t(d[a]) for a in range(3)]
            return P.rollout(*vv, gamma.detach(), base, params, nsteps, every, dts=dts)["vz"]

        fd = float((base["m"] * (vz_at(1) - vz_at(-1)))[mask].sum()) / (2 * eps)
        pred = sum(float((grads[a].cpu().numpy() * d[a]).sum()) for a in range(3))
        assert abs(fd - pred) <= 1e-4 * max(abs(pred), 1e-8), (trial, fd, pred)


def test_rollout_adjoint_sod64_fd_32_directions():
    """Sod split on a 64^3 jittered lattice, 100 FP64 steps (CFL 0.1), checkpoint every 10:
    d/d(v0, gamma) of the x-momentum of particles with x > 48 at the last step,
    checked with central differences (eps = 1e-6) along 32 random directions."""
    w = ci.config3()
    print(f"[case] {w.name} n={w.n}", flush=True)
    params = P.Params.from_workload(w)
    assert params.cfl == 0.1
    base = _base(w, params)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64), device=DEV)
    v0 = [t(w.vx).requires_grad_(True), t(w.vy).requires_grad_(True), t(w.vz).requires_grad_(True)]
    gamma = torch.tensor([1.4], dtype=torch.float64, device=DEV, requires_grad=True)
    info = {}
    out = P.rollout(*v0, gamma, base, params, 100, 10, info=info)
    mask = out["x"].detach() > 48.0
    J = _objective(out, mask, base["m"])
    grads = torch.autograd.grad(J, v0 + [gamma])
    dts = info["dts"]
    dirs = w.fd_dirs
    errs = []
    for k in range(32):
        d = dirs[k]
        dv = [d[a * w.n:(a + 1) * w.n] for a in range(3)]
        dg = d[3 * w.n:]
        eps = 1e-6

        def Jat(sign):
            vv = [v0[a].detach() + sign * eps * t(dv[a]) for a in range(3)]
            gm = gamma.detach() + sign * eps * t(dg)
            o = P.rollout(*vv, gm, base, params, 100, 10, dts=dts)
            return float(_objective(o, mask, base["m"]))

        fd = (Jat(1) - Jat(-1)) / (2 * eps)
        pred = sum(float((grads[a].cpu().numpy() * dv[a]).sum()) for a in range(3)) + \
            float(grads[3].cpu().numpy()[0] * dg[0])
        errs.append(abs(fd - pred) / max(abs(pred), 1e-12))
    print("fd rel errors: max %.2e median %.2e; adjoint/forward %.2f" %
          (max(errs), float(np.median(errs)), info["backward_s"] / info["forward_s"]), flush=True)
    assert max(errs) <= 1e-4, errs


def piston_system(n=8, seed=5):
    """The block moving onto the piston (x_w = 0.2 + 0.4 t): at t = 0.3 the first layers have
    mirror partners, and a step of 0.2 reflects some of the first layer."""
    w = system(n=n, seed=seed)
    w.vx = w.vx - 0.5
    w.wall = (0.2, 0.4)
    return w


def _np_state(g, w):
    s = {k: g[k].cpu().numpy() for k in F8}
    s["m"] = w.m
    s["mat"] = w.mat
    return s


def test_rates_vjp_with_the_piston_matches_autograd():
    """Mirror partners: the GPU VJP of the rates at t against autograd of the FP64 reference
    with the mirror pairs (j's image at 2 x_w - x_j, x-velocity 2 v_w - v_x,j)."""
    w = piston_system()
    t = 0.3
    xw = w.wall[0] + w.wall[1] * t
    params = P.Params.from_workload(w)
    g = P.state_from_workload(w, params, DEV)
    s = _np_state(g, w)
    mir = T.mirror_pairs_of(s, w.kappa * w.h, xw)
    assert len(mir[0]) > 100 and int((mir[0] == mir[1]).sum()) > 10  # self-images among them
    rng = np.random.default_rng(21)
    cot = {k: rng.standard_normal(w.n) for k in ("drho", "dvx", "dvy", "dvz", "dE")}
    gs, ge = P.csph_rates_vjp(g, params, {k: torch.as_tensor(v, device=DEV) for k, v in cot.items()},
                              t=t)
    et, gg, pi = tparams(w, True)
    st = {k: torch.as_tensor(s[k]).clone().requires_grad_(True) for k in F8}
    out = T.rates_torch(st, torch.as_tensor(w.m), torch.as_tensor(w.mat).long(), et, gg, pi,
                        T.pairs_of(O.cfg_for(w), s), w.kappa * w.h, mirror=mir,
                        wall=(xw, w.wall[1]))
    J = sum((o * torch.as_tensor(cot[k])).sum()
            for o, k in zip(out, ("drho", "dvx", "dvy", "dvz", "dE")))
    ref = torch.autograd.grad(J, [st[k] for k in F8] + [gg, pi])
    for a, k in enumerate(F8):
        e = relmax(gs[k].cpu().numpy(), ref[a].numpy())
        assert e <= 1e-10, (k, e)
    ge = ge.cpu().numpy()
    assert relmax(ge[0::2], ref[8].numpy()) <= 1e-10
    assert abs(ge[3] - float(ref[9][1])) <= 1e-10 * abs(float(ref[9][1]))


@pytest.mark.parametrize("seed", [5, 6])
def test_step_vjp_with_the_piston_matches_autograd_and_dot_product(seed):
    """The step with mirror partners at x_w(t) and reflections off x_w(t + dt): the GPU VJP
    against autograd of the FP64 reference (the branch taken at the base state), and the
    dot-product test against the GPU's own forward step."""
    w = piston_system(seed=seed)
    t, dt = 0.3, 0.2
    params = P.Params.from_workload(w, reorder=False)
    g = P.state_from_workload(w, params, DEV)
    s = _np_state(g, w)
    replay = P.Params.from_workload(w, reorder=False, cfl=0.0)

    def fwd(delta=None, eps=0.0):
        tt = {k: g[k] + (eps * torch.as_tensor(delta[k], device=DEV) if delta else 0.0)
              for k in F8}
        tt["m"] = g["m"]
        st2 = P.State(tt, g.mat)
        P.csph_step(st2, replay, P.StepScalars(DEV, t0=t), s_out=st2, dt_in=dt)
        return {k: st2[k].cpu().numpy() for k in F8}

    base = fwd()
    xw1 = w.wall[0] + w.wall[1] * (t + dt)
    assert np.sum(base["vx"] > 0.3) > 3 and np.all(base["x"] >= xw1)  # reflections happened
    rng = np.random.default_rng(seed + 30)
    lam = {k: rng.standard_normal(w.n) for k in F8}
    gn = {k: torch.as_tensor(v, device=DEV).clone() for k, v in lam.items()}
    gp, ge = P.csph_step_vjp(g, params, dt, gn, g_prev={k: torch.empty_like(v) for k, v in gn.items()},
                             t=t)
    et, gg, pi = tparams(w, True)
    st = {k: torch.as_tensor(s[k]).clone().requires_grad_(True) for k in F8}
    mir = T.mirror_pairs_of(s, w.kappa * w.h, w.wall[0] + w.wall[1] * t)
    out = T.step_torch(st, torch.as_tensor(w.m), torch.as_tensor(w.mat).long(), et, gg, pi,
                       T.pairs_of(O.cfg_for(w), s), w.kappa * w.h, dt, mirror=mir, wall=w.wall,
                       t=t)
    for k in F8:  # the reference takes the GPU step's branches
        assert np.abs(out[k].detach().numpy() - base[k]).max() <= 1e-12 * (1 + np.abs(base[k]).max()), k
    J = sum((out[k] * torch.as_tensor(lam[k])).sum() for k in F8)
    ref = torch.autograd.grad(J, [st[k] for k in F8] + [gg, pi])
    for a, k in enumerate(F8):
        assert relmax(gp[k].cpu().numpy(), ref[a].numpy()) <= 1e-10, k
    ge = ge.cpu().numpy()
    assert relmax(ge[0::2], ref[8].numpy()) <= 1e-10
    d = {k: rng.standard_normal(w.n) for k in F8}
    eps = 1e-6
    fp, fm = fwd(d, eps), fwd(d, -eps)
    jvp = sum(float(((fp[k] - fm[k]) / (2 * eps) * lam[k]).sum()) for k in F8)
    vjp = sum(float((gp[k].cpu().numpy() * d[k]).sum()) for k in F8)
    assert abs(jvp - vjp) <= 1e-7 * max(abs(vjp), 1.0), (jvp, vjp)


def test_rollout_with_the_piston_matches_reference_and_fd():
    """Porous 12^3 sample driven by the piston, 10 FP64 CFL steps from t0 = 0.05, checkpoint
    every 4: d/d(v0, gamma) of the x-momentum of the particles beyond the middle against the
    FP64 CPU reference (autograd over the same dt sequence, mirror pairs and reflections) and
    central differences of the GPU forward."""
    w = ci.config2(nside=12)
    print(f"[case] piston rollout n={w.n}", flush=True)
    params = P.Params.from_workload(w, cfl=0.3)
    base = _base(w, params)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64), device=DEV)
    v0 = [t(w.vx).requires_grad_(True), t(w.vy).requires_grad_(True), t(w.vz).requires_grad_(True)]
    gamma = torch.tensor([e[1] for e in w.eos], dtype=torch.float64, device=DEV,
                         requires_grad=True)
    nsteps, every, t0 = 10, 4, 0.05
    info = {}
    P.rollout(*v0, gamma, base, params, nsteps, every, info=info, t0=t0)
    dts = info["dts"]
    out = P.rollout(*v0, gamma, base, params, nsteps, every, dts=dts, t0=t0)
    xmid = float(np.median(w.x))
    mask = out["x"].detach() > xmid
    J = _objective(out, mask, base["m"])
    grads = torch.autograd.grad(J, v0 + [gamma])
    # FP64 CPU reference over the same steps: mirror pairs at each step's start time
    cfg = O.cfg_for(w)
    et, gg, pi = tparams(w, True)
    gg = gg.clone().detach().requires_grad_(True)
    mat = torch.as_tensor(w.mat).long()
    m = torch.as_tensor(w.m)
    vr = [torch.as_tensor(a).clone().requires_grad_(True) for a in (w.vx, w.vy, w.vz)]
    E0 = T.init_energy_torch(torch.as_tensor(w.rho), torch.as_tensor(w.p), *vr, mat, et, gg, pi)
    st = {"x": torch.as_tensor(w.x), "y": torch.as_tensor(w.y), "z": torch.as_tensor(w.z),
          "vx": vr[0], "vy": vr[1], "vz": vr[2], "rho": torch.as_tensor(w.rho), "E": E0}
    H = w.kappa * w.h
    tk = t0
    nmir = 0
    for k in range(nsteps):
        sn = {kk: st[kk].detach().numpy() for kk in ("x", "y", "z")}
        mir = T.mirror_pairs_of(sn, H, w.wall[0] + w.wall[1] * tk)
        nmir += len(mir[0])
        st = T.step_torch(st, m, mat, et, gg, pi, T.pairs_of(cfg, sn), H, dts[k], mirror=mir,
                          wall=w.wall, t=tk)
        tk = tk + dts[k]
    assert nmir > 1000
    mref = st["x"].detach() > xmid
    assert torch.equal(mref, mask.cpu())
    Jr = (st["vx"][mref] * m[mref]).sum()
    ref = torch.autograd.grad(Jr, vr + [gg])
    assert abs(float(J.detach()) - float(Jr.detach())) <= 1e-11 * abs(float(Jr.detach()))
    for a in range(3):
        assert relmax(grads[a].cpu().numpy(), ref[a].numpy()) <= 1e-9, a
    assert relmax(grads[3].cpu().numpy(), ref[3].numpy()) <= 1e-9
    rng = np.random.default_rng(13)
    for trial in range(4):
        d = [rng.standard_normal(w.n) for _ in range(3)]
        dg = rng.standard_normal(len(w.eos))
        eps = 1e-6

        def Jat(sign):
            vv = [v0[a].detach() + sign * eps * t(d[a]) for a in range(3)]
            gm = gamma.detach() + sign * eps * t(dg)
            o = P.rollout(*vv, gm, base, params, nsteps, every, dts=dts, t0=t0)
            return float(_objective(o, mask, base["m"]))

        fd = (Jat(1) - Jat(-1)) / (2 * eps)
        pred = sum(float((grads[a].cpu().numpy() * d[a]).sum()) for a in range(3)) + \
            float((grads[3].cpu().numpy() * dg).sum())
        assert abs(fd - pred) <= 1e-4 * max(abs(pred), 1e-8), (trial, fd, pred)


def mg_system(n=8, seed=7):
    """An ideal gas and a Mie-Grueneisen solid (aluminium-like constants) side by side, the
    solid compressed by 0-8 % or expanded by up to 3 % against rho0."""
    w = system(n=n, seed=seed)
    rng = np.random.default_rng(seed + 1)
    solid = w.mat == 1
    w.rho = np.where(solid, ci.MG_ALUMINIUM[3] * rng.uniform(0.97, 1.08, w.n), w.rho)
    w.m = w.rho.copy()
    w.eos = [(0, 1.4, 0.0), ci.MG_ALUMINIUM]
    return w


def test_rates_and_step_vjp_with_mie_grueneisen_match_autograd():
    """The EOS chain through the Mie-Grueneisen pressure and sound speed (forward-mode partials
    on the GPU) against autograd of the FP64 reference; d/dGamma in the gamma slot, 0 in the
    p_inf slot of the solid."""
    w = mg_system()
    params = P.Params.from_workload(w, reorder=False)
    g = P.state_from_workload(w, params, DEV)
    s = _np_state(g, w)
    et = list(w.eos)
    rng = np.random.default_rng(22)
    cot = {k: rng.standard_normal(w.n) for k in ("drho", "dvx", "dvy", "dvz", "dE")}
    gs, ge = P.csph_rates_vjp(g, params, {k: torch.as_tensor(v, device=DEV) for k, v in cot.items()})
    _, gg, pi = tparams(w, True)
    st = {k: torch.as_tensor(s[k]).clone().requires_grad_(True) for k in F8}
    pairs = T.pairs_of(O.cfg_for(w), s)
    out = T.rates_torch(st, torch.as_tensor(w.m), torch.as_tensor(w.mat).long(), et, gg, pi,
                        pairs, w.kappa * w.h)
    J = sum((o * torch.as_tensor(cot[k])).sum()
            for o, k in zip(out, ("drho", "dvx", "dvy", "dvz", "dE")))
    ref = torch.autograd.grad(J, [st[k] for k in F8] + [gg])
    for a, k in enumerate(F8):
        assert relmax(gs[k].cpu().numpy(), ref[a].numpy()) <= 1e-10, k
    ge = ge.cpu().numpy()
    assert relmax(ge[0::2], ref[8].numpy()) <= 1e-10
    assert ge[3] == 0.0
    dt = 0.02
    lam = {k: rng.standard_normal(w.n) for k in F8}
    gn = {k: torch.as_tensor(v, device=DEV).clone() for k, v in lam.items()}
    gp, ge = P.csph_step_vjp(g, params, dt, gn, g_prev={k: torch.empty_like(v) for k, v in gn.items()})
    st = {k: torch.as_tensor(s[k]).clone().requires_grad_(True) for k in F8}
    out = T.step_torch(st, torch.as_tensor(w.m), torch.as_tensor(w.mat).long(), et, gg, pi,
                       pairs, w.kappa * w.h, dt)
    J = sum((out[k] * torch.as_tensor(lam[k])).sum() for k in F8)
    ref = torch.autograd.grad(J, [st[k] for k in F8] + [gg])
    for a, k in enumerate(F8):
        assert relmax(gp[k].cpu().numpy(), ref[a].numpy()) <= 1e-10, k
    assert relmax(ge.cpu().numpy()[0::2], ref[8].numpy()) <= 1e-10


def test_init_energy_vjp_with_mie_grueneisen_matches_autograd():
    w = mg_system(seed=9)
    w.p = np.where(w.mat == 1, np.random.default_rng(9).uniform(-0.5, 3.0, w.n), w.p)
    params = P.Params.from_workload(w)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64), device=DEV)
    gE = np.random.default_rng(10).standard_normal(w.n)
    gv = [torch.zeros(w.n, dtype=torch.float64, device=DEV) for _ in range(3)]
    grho = torch.zeros(w.n, dtype=torch.float64, device=DEV)
    geos = torch.zeros(4, dtype=torch.float64, device=DEV)
    P.csph_init_energy_vjp(t(w.rho), t(w.p), t(w.vx), t(w.vy), t(w.vz),
                           torch.as_tensor(w.mat, device=DEV), params, t(gE), g_v=gv, g_rho=grho,
                           g_eos=geos)
    _, gg, pi = tparams(w, True)
    vx = torch.as_tensor(w.vx).clone().requires_grad_(True)
    rho = torch.as_tensor(w.rho).clone().requires_grad_(True)
    E = T.init_energy_torch(rho, torch.as_tensor(w.p), vx, torch.as_tensor(w.vy),
                            torch.as_tensor(w.vz), torch.as_tensor(w.mat).long(), list(w.eos),
                            gg, pi)
    ref = torch.autograd.grad((E * torch.as_tensor(gE)).sum(), [vx, rho, gg])
    assert relmax(gv[0].cpu().numpy(), ref[0].numpy()) <= 1e-13
    assert relmax(grho.cpu().numpy(), ref[1].numpy()) <= 1e-12
    assert relmax(geos.cpu().numpy()[0::2], ref[2].numpy()) <= 1e-12
    assert geos.cpu().numpy()[3] == 0.0


def test_rollout_plate_impact_mie_grueneisen_reference_and_fd():
    """Aluminium plate onto lead (8 x 8 x 4 lattices each, Mie-Grueneisen), 12 FP64 CFL steps,
    checkpoint every 5: d/d(v0, Gamma) of the z-momentum of the aluminium against the FP64 CPU
    reference (autograd over the same dt sequence) and central differences of the GPU
    forward."""
    w = ci.mg_plates(8, 8, 4, gap=2.0, v_impact=0.5, seed=3)
    print(f"[case] mg plates rollout n={w.n}", flush=True)
    params = P.Params.from_workload(w, cfl=0.3)
    base = _base(w, params)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64), device=DEV)
    v0 = [t(w.vx).requires_grad_(True), t(w.vy).requires_grad_(True), t(w.vz).requires_grad_(True)]
    gamma = torch.tensor([e[1] for e in w.eos], dtype=torch.float64, device=DEV,
                         requires_grad=True)
    nsteps, every = 12, 5
    info = {}
    P.rollout(*v0, gamma, base, params, nsteps, every, info=info)
    dts = info["dts"]
    out = P.rollout(*v0, gamma, base, params, nsteps, every, dts=dts)
    mask = torch.as_tensor(w.mat == 1, device=DEV)
    J = (out["vz"][mask] * base["m"][mask]).sum()
    grads = torch.autograd.grad(J, v0 + [gamma])
    cfg = O.cfg_for(w)
    _, gg, pi = tparams(w, True)
    gg = gg.clone().detach().requires_grad_(True)
    mat = torch.as_tensor(w.mat).long()
    m = torch.as_tensor(w.m)
    vr = [torch.as_tensor(a).clone().requires_grad_(True) for a in (w.vx, w.vy, w.vz)]
    E0 = T.init_energy_torch(torch.as_tensor(w.rho), torch.as_tensor(w.p), *vr, mat,
                             list(w.eos), gg, pi)
    st = {"x": torch.as_tensor(w.x), "y": torch.as_tensor(w.y), "z": torch.as_tensor(w.z),
          "vx": vr[0], "vy": vr[1], "vz": vr[2], "rho": torch.as_tensor(w.rho), "E": E0}
    for k in range(nsteps):
        pairs = T.pairs_of(cfg, {kk: st[kk].detach().numpy() for kk in ("x", "y", "z")})
        st = T.step_torch(st, m, mat, list(w.eos), gg, pi, pairs, w.kappa * w.h, dts[k])
    mref = torch.as_tensor(w.mat == 1)
    Jr = (st["vz"][mref] * m[mref]).sum()
    ref = torch.autograd.grad(Jr, vr + [gg])
    assert abs(float(J.detach()) - float(Jr.detach())) <= 1e-11 * abs(float(Jr.detach()))
    for a in range(3):
        assert relmax(grads[a].cpu().numpy(), ref[a].numpy()) <= 1e-9, a
    assert relmax(grads[3].cpu().numpy(), ref[3].numpy()) <= 1e-9
    assert float(np.abs(ref[3].numpy()).min()) > 0.0  # both Gammas matter
    rng = np.random.default_rng(17)
    for trial in range(4):
        d = [rng.standard_normal(w.n) for _ in range(3)]
        dg = rng.standard_normal(len(w.eos))
        eps = 1e-6

        def Jat(sign):
            vv = [v0[a].detach() + sign * eps * t(d[a]) for a in range(3)]
            gm = gamma.detach() + sign * eps * t(dg)
            o = P.rollout(*vv, gm, base, params, nsteps, every, dts=dts)
            return float((o["vz"][mask] * base["m"][mask]).sum())

        fd = (Jat(1) - Jat(-1)) / (2 * eps)
        pred = sum(float((grads[a].cpu().numpy() * d[a]).sum()) for a in range(3)) + \
            float((grads[3].cpu().numpy() * dg).sum())
        assert abs(fd - pred) <= 1e-4 * max(abs(pred), 1e-8), (trial, fd, pred)


@pytest.mark.parametrize("periodic,wall", [(7, None), (5, None), (6, (0.2, 0.4))],
                         ids=["xyz", "xz", "yz+piston"])
def test_rates_and_step_vjp_periodic_match_autograd(periodic, wall):
    """Image partners (and, with the piston on periodic sides, mirror partners through the
    images): the GPU VJPs of the rates at t and of a step that carries particles through the
    faces, against autograd of the FP64 reference, and the dot-product test against the GPU's
    own forward step.  Periodic x with an open y hands the kernels the axes exchanged."""
    from test_adjoint_ref import periodic_system
    w = periodic_system(periodic, seed=12, wall=wall)
    print(f"[case] periodic vjp {periodic} wall={wall} n={w.n}", flush=True)
    t, dt = 0.3, 0.2
    H = w.kappa * w.h
    params = P.Params.from_workload(w, reorder=False)
    g = P.state_from_workload(w, params, DEV)
    s = _np_state(g, w)
    cfg = O.cfg_for(w)
    pairs = T.pairs_of(cfg, s)
    mir, wt = None, None
    if wall is not None:
        mir = T.mirror_pairs_of(s, H, wall[0] + wall[1] * t, box=w.box, periodic=periodic)
        wt = (wall[0] + wall[1] * t, wall[1])
    et, gg, pi = tparams(w, True)
    m, mat = torch.as_tensor(w.m), torch.as_tensor(w.mat).long()
    rng = np.random.default_rng(periodic + 60)
    cot = {k: rng.standard_normal(w.n) for k in ("drho", "dvx", "dvy", "dvz", "dE")}
    gs, ge = P.csph_rates_vjp(g, params, {k: torch.as_tensor(v, device=DEV) for k, v in cot.items()},
                              t=t)
    st = {k: torch.as_tensor(s[k]).clone().requires_grad_(True) for k in F8}
    out = T.rates_torch(st, m, mat, et, gg, pi, pairs, H, mirror=mir, wall=wt)
    J = sum((o * torch.as_tensor(cot[k])).sum()
            for o, k in zip(out, ("drho", "dvx", "dvy", "dvz", "dE")))
    ref = torch.autograd.grad(J, [st[k] for k in F8] + [gg, pi])
    for a, k in enumerate(F8):
        assert relmax(gs[k].cpu().numpy(), ref[a].numpy()) <= 1e-10, ("rates", k)
    assert relmax(ge.cpu().numpy()[0::2], ref[8].numpy()) <= 1e-10
    # the step
    replay = P.Params.from_workload(w, reorder=False, cfl=0.0)

    def fwd(delta=None, eps=0.0):
        tt = {k: g[k] + (eps * torch.as_tensor(delta[k], device=DEV) if delta else 0.0)
              for k in F8}
        tt["m"] = g["m"]
        st2 = P.State(tt, g.mat)
        P.csph_step(st2, replay, P.StepScalars(DEV, t0=t), s_out=st2, dt_in=dt)
        return {k: st2[k].cpu().numpy() for k in F8}

    base = fwd()
    crossed = sum(int(np.sum(np.abs(base[k] - s[k]) > 4.0)) for a, k in enumerate("xyz")
                  if (periodic >> a) & 1)
    assert crossed > 3  # particles crossed a face
    lam = {k: rng.standard_normal(w.n) for k in F8}
    gn = {k: torch.as_tensor(v, device=DEV).clone() for k, v in lam.items()}
    gp, ge = P.csph_step_vjp(g, params, dt, gn, g_prev={k: torch.empty_like(v) for k, v in gn.items()},
                             t=t)
    st = {k: torch.as_tensor(s[k]).clone().requires_grad_(True) for k in F8}
    out = T.step_torch(st, m, mat, et, gg, pi, pairs, H, dt, mirror=mir, wall=wall, t=t,
                       box=w.box, periodic=periodic)
    for k in F8:
        assert np.abs(out[k].detach().numpy() - base[k]).max() <= 1e-12 * (1 + np.abs(base[k]).max()), k
    J = sum((out[k] * torch.as_tensor(lam[k])).sum() for k in F8)
    ref = torch.autograd.grad(J, [st[k] for k in F8] + [gg, pi])
    for a, k in enumerate(F8):
        assert relmax(gp[k].cpu().numpy(), ref[a].numpy()) <= 1e-10, ("step", k)
    d = {k: rng.standard_normal(w.n) for k in F8}
    eps = 1e-6
    fp, fm = fwd(d, eps), fwd(d, -eps)
    jvp = sum(float(((fp[k] - fm[k]) / (2 * eps) * lam[k]).sum()) for k in F8)
    vjp = sum(float((gp[k].cpu().numpy() * d[k]).sum()) for k in F8)
    assert abs(jvp - vjp) <= 1e-7 * max(abs(vjp), 1.0), (jvp, vjp)


def test_rollout_periodic_box_reference_and_fd():
    """A closed periodic box (8 x 9 x 8), 10 FP64 CFL steps with particles crossing the faces,
    checkpoint every 4: d/d(v0, gamma) of the x-momentum of the particles in the upper half
    (in z) at the end, against the FP64 CPU reference and central differences of the GPU
    forward."""
    w = ci.periodic_block(8, 9, 8, seed=14, periodic=7, amp=0.3)
    rng = np.random.default_rng(14)
    w.vx, w.vy, w.vz = (rng.uniform(-0.6, 0.6, w.n) for _ in range(3))
    w.vy = w.vy + 1.0
    w.p = rng.uniform(0.5, 1.5, w.n)
    params = P.Params.from_workload(w, cfl=0.3)
    base = _base(w, params)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64), device=DEV)
    v0 = [t(w.vx).requires_grad_(True), t(w.vy).requires_grad_(True), t(w.vz).requires_grad_(True)]
    gamma = torch.tensor([e[1] for e in w.eos], dtype=torch.float64, device=DEV,
                         requires_grad=True)
    nsteps, every = 10, 4
    info = {}
    P.rollout(*v0, gamma, base, params, nsteps, every, info=info)
    dts = info["dts"]
    out = P.rollout(*v0, gamma, base, params, nsteps, every, dts=dts)
    mask = out["z"].detach() > 4.0
    J = _objective(out, mask, base["m"])
    grads = torch.autograd.grad(J, v0 + [gamma])
    cfg = O.cfg_for(w)
    et, gg, pi = tparams(w, True)
    gg = gg.clone().detach().requires_grad_(True)
    mat = torch.as_tensor(w.mat).long()
    m = torch.as_tensor(w.m)
    vr = [torch.as_tensor(a).clone().requires_grad_(True) for a in (w.vx, w.vy, w.vz)]
    E0 = T.init_energy_torch(torch.as_tensor(w.rho), torch.as_tensor(w.p), *vr, mat, et, gg, pi)
    st = {"x": torch.as_tensor(w.x), "y": torch.as_tensor(w.y), "z": torch.as_tensor(w.z),
          "vx": vr[0], "vy": vr[1], "vz": vr[2], "rho": torch.as_tensor(w.rho), "E": E0}
    y0 = w.y.copy()
    for k in range(nsteps):
        pairs = T.pairs_of(cfg, {kk: st[kk].detach().numpy() for kk in ("x", "y", "z")})
        st = T.step_torch(st, m, mat, et, gg, pi, pairs, w.kappa * w.h, dts[k], box=w.box,
                          periodic=7)
    assert np.sum(st["y"].detach().numpy() < y0 - 4.0) > 10  # wrapped through the top face
    mref = st["z"].detach() > 4.0
    assert torch.equal(mref, mask.cpu())
    Jr = (st["vx"][mref] * m[mref]).sum()
    ref = torch.autograd.grad(Jr, vr + [gg])
    assert abs(float(J.detach()) - float(Jr.detach())) <= 1e-11 * max(abs(float(Jr.detach())), 1e-3)
    for a in range(3):
        assert relmax(grads[a].cpu().numpy(), ref[a].numpy()) <= 1e-9, a
    assert relmax(grads[3].cpu().numpy(), ref[3].numpy()) <= 1e-9
    for trial in range(4):
        d = [rng.standard_normal(w.n) for _ in range(3)]
        dg = rng.standard_normal(len(w.eos))
        eps = 1e-6

        def Jat(sign):
            vv = [v0[a].detach() + sign * eps * t(d[a]) for a in range(3)]
            gm = gamma.detach() + sign * eps * t(dg)
            o = P.rollout(*vv, gm, base, params, nsteps, every, dts=dts)
            return float(_objective(o, mask, base["m"]))

        fd = (Jat(1) - Jat(-1)) / (2 * eps)
        pred = sum(float((grads[a].cpu().numpy() * d[a]).sum()) for a in range(3)) + \
            float((grads[3].cpu().numpy() * dg).sum())
        assert abs(fd - pred) <= 1e-4 * max(abs(pred), 1e-8), (trial, fd, pred)


@pytest.mark.parametrize("wall", [None, (0.2, 0.4)], ids=["open", "piston"])
def test_rates_and_step_vjp_pair_h_match_autograd(wall):
    """Pair-h mode (each pair's support kappa (d_i + d_j)/2, kappa = 1.936, d held fixed): the
    GPU VJPs of the rates and of the step against autograd of the FP64 reference, and the
    dot-product test against the GPU's own forward step."""
    w = system(n=8, seed=23)
    rng = np.random.default_rng(23)
    d = rng.uniform(0.8, 1.3, w.n)
    if wall is not None:
        w.vx = w.vx - 0.5
        w.wall = wall
    print(f"[case] pair-h vjp wall={wall} n={w.n}", flush=True)
    t, dt = 0.3, 0.1
    params = P.Params.from_workload(w, reorder=False, h_mode="pair", kappa=1.936, cell_size=0.0)
    g = P.state_from_workload(w, params, DEV)
    g.d = torch.as_tensor(d, device=DEV)
    s = _np_state(g, w)
    s["d"] = d
    ph = (1.936, d)
    cfg = O.cfg_for(w, h_mode=1, kappa=1.936)
    pairs = T.pairs_of(cfg, s)
    mir, wt = None, None
    if wall is not None:
        mir = T.mirror_pairs_of(s, 0.0, wall[0] + wall[1] * t, pair_h=ph)
        wt = (wall[0] + wall[1] * t, wall[1])
    et, gg, pi = tparams(w, True)
    m, mat = torch.as_tensor(w.m), torch.as_tensor(w.mat).long()
    cot = {k: rng.standard_normal(w.n) for k in ("drho", "dvx", "dvy", "dvz", "dE")}
    gs, ge = P.csph_rates_vjp(g, params, {k: torch.as_tensor(v, device=DEV) for k, v in cot.items()},
                              t=t)
    st = {k: torch.as_tensor(s[k]).clone().requires_grad_(True) for k in F8}
    out = T.rates_torch(st, m, mat, et, gg, pi, pairs, 0.0, mirror=mir, wall=wt, pair_h=ph)
    J = sum((o * torch.as_tensor(cot[k])).sum()
            for o, k in zip(out, ("drho", "dvx", "dvy", "dvz", "dE")))
    ref = torch.autograd.grad(J, [st[k] for k in F8] + [gg, pi])
    for a, k in enumerate(F8):
        assert relmax(gs[k].cpu().numpy(), ref[a].numpy()) <= 1e-10, ("rates", k)
    assert relmax(ge.cpu().numpy()[0::2], ref[8].numpy()) <= 1e-10
    replay = P.Params.from_workload(w, reorder=False, h_mode="pair", kappa=1.936, cell_size=0.0,
                                    cfl=0.0)

    def fwd(delta=None, eps=0.0):
        tt = {k: g[k] + (eps * torch.as_tensor(delta[k], device=DEV) if delta else 0.0)
              for k in F8}
        tt["m"] = g["m"]
        st2 = P.State(tt, g.mat, g.d)
        P.csph_step(st2, replay, P.StepScalars(DEV, t0=t), s_out=st2, dt_in=dt)
        return {k: st2[k].cpu().numpy() for k in F8}

    base = fwd()
    lam = {k: rng.standard_normal(w.n) for k in F8}
    gn = {k: torch.as_tensor(v, device=DEV).clone() for k, v in lam.items()}
    gp, ge = P.csph_step_vjp(g, params, dt, gn, g_prev={k: torch.empty_like(v) for k, v in gn.items()},
                             t=t)
    st = {k: torch.as_tensor(s[k]).clone().requires_grad_(True) for k in F8}
    out = T.step_torch(st, m, mat, et, gg, pi, pairs, 0.0, dt, mirror=mir, wall=wall, t=t,
                       pair_h=ph)
    for k in F8:
        assert np.abs(out[k].detach().numpy() - base[k]).max() <= 1e-12 * (1 + np.abs(base[k]).max()), k
    J = sum((out[k] * torch.as_tensor(lam[k])).sum() for k in F8)
    ref = torch.autograd.grad(J, [st[k] for k in F8] + [gg, pi])
    for a, k in enumerate(F8):
        assert relmax(gp[k].cpu().numpy(), ref[a].numpy()) <= 1e-10, ("step", k)
    dd = {k: rng.standard_normal(w.n) for k in F8}
    eps = 1e-6
    fp, fm = fwd(dd, eps), fwd(dd, -eps)
    jvp = sum(float(((fp[k] - fm[k]) / (2 * eps) * lam[k]).sum()) for k in F8)
    vjp = sum(float((gp[k].cpu().numpy() * dd[k]).sum()) for k in F8)
    assert abs(jvp - vjp) <= 1e-7 * max(abs(vjp), 1.0), (jvp, vjp)


def test_rates_and_step_vjp_pair_h_periodic_piston_match_autograd():
    """Pair-h mode on periodic sides with the piston (pair supports, image partners, mirror
    partners through the images, reflections and the wrap): the GPU VJPs of the rates and of
    the step against autograd of the FP64 reference, and the dot-product test against the
    GPU's own forward step."""
    from test_adjoint_ref import periodic_system
    w = periodic_system(6, seed=13, wall=(0.2, 0.4))
    d = np.random.default_rng(14).uniform(0.8, 1.3, w.n)
    print(f"[case] pair-h periodic piston vjp n={w.n}", flush=True)
    t, dt = 0.3, 0.2
    params = P.Params.from_workload(w, reorder=False, h_mode="pair", kappa=1.936, cell_size=0.0)
    g = P.state_from_workload(w, params, DEV)
    g.d = torch.as_tensor(d, device=DEV)
    s = _np_state(g, w)
    s["d"] = d
    ph = (1.936, d)
    cfg = O.cfg_for(w, h_mode=1, kappa=1.936)
    pairs = T.pairs_of(cfg, s)
    mir = T.mirror_pairs_of(s, 0.0, 0.2 + 0.4 * t, box=w.box, periodic=6, pair_h=ph)
    wt = (0.2 + 0.4 * t, 0.4)
    et, gg, pi = tparams(w, True)
    m, mat = torch.as_tensor(w.m), torch.as_tensor(w.mat).long()
    rng = np.random.default_rng(66)
    cot = {k: rng.standard_normal(w.n) for k in ("drho", "dvx", "dvy", "dvz", "dE")}
    gs, ge = P.csph_rates_vjp(g, params, {k: torch.as_tensor(v, device=DEV) for k, v in cot.items()},
                              t=t)
    st = {k: torch.as_tensor(s[k]).clone().requires_grad_(True) for k in F8}
    out = T.rates_torch(st, m, mat, et, gg, pi, pairs, 0.0, mirror=mir, wall=wt, pair_h=ph)
    J = sum((o * torch.as_tensor(cot[k])).sum()
            for o, k in zip(out, ("drho", "dvx", "dvy", "dvz", "dE")))
    ref = torch.autograd.grad(J, [st[k] for k in F8] + [gg, pi])
    for a, k in enumerate(F8):
        assert relmax(gs[k].cpu().numpy(), ref[a].numpy()) <= 1e-10, ("rates", k)
    assert relmax(ge.cpu().numpy()[0::2], ref[8].numpy()) <= 1e-10
    replay = P.Params.from_workload(w, reorder=False, h_mode="pair", kappa=1.936, cell_size=0.0,
                                    cfl=0.0)

    def fwd(delta=None, eps=0.0):
        tt = {k: g[k] + (eps * torch.as_tensor(delta[k], device=DEV) if delta else 0.0)
              for k in F8}
        tt["m"] = g["m"]
        st2 = P.State(tt, g.mat, g.d)
        P.csph_step(st2, replay, P.StepScalars(DEV, t0=t), s_out=st2, dt_in=dt)
        return {k: st2[k].cpu().numpy() for k in F8}

    base = fwd()
    crossed = sum(int(np.sum(np.abs(base[k] - s[k]) > 4.0)) for k in ("y", "z"))
    assert crossed > 3  # particles crossed a periodic face
    lam = {k: rng.standard_normal(w.n) for k in F8}
    gn = {k: torch.as_tensor(v, device=DEV).clone() for k, v in lam.items()}
    gp, ge = P.csph_step_vjp(g, params, dt, gn, g_prev={k: torch.empty_like(v) for k, v in gn.items()},
                             t=t)
    st = {k: torch.as_tensor(s[k]).clone().requires_grad_(True) for k in F8}
    out = T.step_torch(st, m, mat, et, gg, pi, pairs, 0.0, dt, mirror=mir, wall=w.wall, t=t,
                       box=w.box, periodic=6, pair_h=ph)
    for k in F8:
        assert np.abs(out[k].detach().numpy() - base[k]).max() <= 1e-12 * (1 + np.abs(base[k]).max()), k
    J = sum((out[k] * torch.as_tensor(lam[k])).sum() for k in F8)
    ref = torch.autograd.grad(J, [st[k] for k in F8] + [gg, pi])
    for a, k in enumerate(F8):
        assert relmax(gp[k].cpu().numpy(), ref[a].numpy()) <= 1e-10, ("step", k)
    dd = {k: rng.standard_normal(w.n) for k in F8}
    eps = 1e-6
    fp, fm = fwd(dd, eps), fwd(dd, -eps)
    jvp = sum(float(((fp[k] - fm[k]) / (2 * eps) * lam[k]).sum()) for k in F8)
    vjp = sum(float((gp[k].cpu().numpy() * dd[k]).sum()) for k in F8)
    assert abs(jvp - vjp) <= 1e-7 * max(abs(vjp), 1.0), (jvp, vjp)


def test_rollout_paper_mode_plates_reference_and_fd():
    """The paper's material mode on a small plate impact: aluminium onto lead (8 x 8 x 4 each,
    Mie-Grueneisen), pair-h support with kappa = 1.936 and sizes d of 0.95-1.15 held fixed,
    12 FP64 CFL steps, checkpoint every 5: d/d(v0, Gamma) of the aluminium's z-momentum against
    the FP64 CPU reference and central differences of the GPU forward."""
    w = ci.mg_plates(8, 8, 4, gap=1.5, v_impact=0.5, seed=4)
    d = np.random.default_rng(4).uniform(0.95, 1.15, w.n)
    print(f"[case] paper-mode plates rollout n={w.n}", flush=True)
    params = P.Params.from_workload(w, cfl=0.3, h_mode="pair", kappa=1.936, cell_size=0.0)
    base = _base(w, params)
    base["d"] = torch.as_tensor(d, device=DEV)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64), device=DEV)
    v0 = [t(w.vx).requires_grad_(True), t(w.vy).requires_grad_(True), t(w.vz).requires_grad_(True)]
    gamma = torch.tensor([e[1] for e in w.eos], dtype=torch.float64, device=DEV,
                         requires_grad=True)
    nsteps, every = 12, 5
    info = {}
    P.rollout(*v0, gamma, base, params, nsteps, every, info=info)
    dts = info["dts"]
    out = P.rollout(*v0, gamma, base, params, nsteps, every, dts=dts)
    mask = torch.as_tensor(w.mat == 1, device=DEV)
    J = (out["vz"][mask] * base["m"][mask]).sum()
    grads = torch.autograd.grad(J, v0 + [gamma])
    cfg = O.cfg_for(w, h_mode=1, kappa=1.936)
    _, gg, pi = tparams(w, True)
    gg = gg.clone().detach().requires_grad_(True)
    mat = torch.as_tensor(w.mat).long()
    m = torch.as_tensor(w.m)
    vr = [torch.as_tensor(a).clone().requires_grad_(True) for a in (w.vx, w.vy, w.vz)]
    E0 = T.init_energy_torch(torch.as_tensor(w.rho), torch.as_tensor(w.p), *vr, mat,
                             list(w.eos), gg, pi)
    st = {"x": torch.as_tensor(w.x), "y": torch.as_tensor(w.y), "z": torch.as_tensor(w.z),
          "vx": vr[0], "vy": vr[1], "vz": vr[2], "rho": torch.as_tensor(w.rho), "E": E0}
    npairs = 0
    for k in range(nsteps):
        sn = {kk: st[kk].detach().numpy() for kk in ("x", "y", "z")}
        sn["d"] = d
        pairs = T.pairs_of(cfg, sn)
        npairs += len(pairs[0])
        st = T.step_torch(st, m, mat, list(w.eos), gg, pi, pairs, 0.0, dts[k],
                          pair_h=(1.936, d))
    assert npairs > 12 * 4 * w.n  # a few partners each within kappa (d_i + d_j)/2
    mref = torch.as_tensor(w.mat == 1)
    Jr = (st["vz"][mref] * m[mref]).sum()
    ref = torch.autograd.grad(Jr, vr + [gg])
    assert abs(float(J.detach()) - float(Jr.detach())) <= 1e-11 * abs(float(Jr.detach()))
    for a in range(3):
        assert relmax(grads[a].cpu().numpy(), ref[a].numpy()) <= 1e-9, a
    assert relmax(grads[3].cpu().numpy(), ref[3].numpy()) <= 1e-9
    rng = np.random.default_rng(19)
    for trial in range(4):
        dv = [rng.standard_normal(w.n) for _ in range(3)]
        dg = rng.standard_normal(len(w.eos))
        eps = 1e-6

        def Jat(sign):
            vv = [v0[a].detach() + sign * eps * t(dv[a]) for a in range(3)]
            gm = gamma.detach() + sign * eps * t(dg)
            o = P.rollout(*vv, gm, base, params, nsteps, every, dts=dts)
            return float((o["vz"][mask] * base["m"][mask]).sum())

        fd = (Jat(1) - Jat(-1)) / (2 * eps)
        pred = sum(float((grads[a].cpu().numpy() * dv[a]).sum()) for a in range(3)) + \
            float((grads[3].cpu().numpy() * dg).sum())
        assert abs(fd - pred) <= 1e-4 * max(abs(pred), 1e-8), (trial, fd, pred)


def _cfl_case(name):
    """(workload, t, extra Params fields, pair_h or None)"""
    from test_adjoint_ref import periodic_system
    if name == "gas":
        return system(n=8, seed=41), 0.0, {}, None
    if name == "piston":
        return piston_system(seed=42), 0.3, {}, None
    if name == "mg":
        return mg_system(seed=43), 0.0, {}, None
    if name == "expanding":  # the density-change limit binds
        w = system(n=8, seed=44)
        for k in ("x", "y", "z"):
            v = getattr(w, k)
            setattr(w, "v" + k, 2.0 * (v - v.mean()))
        return w, 0.0, {}, None
    if name == "periodic":
        return periodic_system(7, seed=45), 0.0, {}, None
    w = system(n=8, seed=46)  # pair h
    d = np.random.default_rng(46).uniform(0.8, 1.3, w.n)
    return w, 0.0, dict(h_mode="pair", kappa=1.936, cell_size=0.0), d


@pytest.mark.parametrize("name", ["gas", "piston", "mg", "expanding", "periodic", "pair-h"])
def test_step_vjp_cfl_matches_autograd_and_dot_product(name):
    """The CFL step's adjoint (csph_step_vjp_cfl): dt recomputed in FP64 equals the GPU step's
    and the oracle's; the gradient, with dt's dependence on the state and the EOS parameters
    (the Courant limit through the signal speed's maximum, or the density-change limit),
    against autograd of the FP64 reference; the dot-product test against the GPU's own CFL
    steps, dt recomputed on every perturbed state."""
    w, t, extra, d = _cfl_case(name)
    print(f"[case] cfl vjp {name} n={w.n}", flush=True)
    params = P.Params.from_workload(w, reorder=False, cfl=0.3, **extra)
    g = P.state_from_workload(w, params, DEV)
    if d is not None:
        g.d = torch.as_tensor(d, device=DEV)
    s = _np_state(g, w)
    H = w.kappa * w.h
    hmode = dict(h_mode=1, kappa=1.936) if d is not None else {}
    cfg = O.cfg_for(w, cfl=0.3, **hmode)
    if d is not None:
        s["d"] = d
    ph = None if d is None else (1.936, d)

    def fwd(delta=None, eps=0.0):
        tt = {k: g[k] + (eps * torch.as_tensor(delta[k], device=DEV) if delta else 0.0)
              for k in F8}
        tt["m"] = g["m"]
        st2 = P.State(tt, g.mat, g.d)
        sc = P.StepScalars(DEV, t0=t)
        P.csph_step(st2, params, sc, s_out=st2)
        return {k: st2[k].cpu().numpy() for k in F8}, float(sc.dt.item())

    base, dt_gpu = fwd()
    rng = np.random.default_rng(90)
    lam = {k: rng.standard_normal(w.n) for k in F8}
    gn = {k: torch.as_tensor(v, device=DEV).clone() for k, v in lam.items()}
    gp, ge, dt = P.csph_step_vjp_cfl(g, params, gn, g_prev={k: torch.empty_like(v) for k, v in gn.items()},
                                     t=t)
    assert dt == dt_gpu
    _, _, dt_o, _ = O.step(cfg, s, t, d=d)
    assert abs(dt - dt_o) <= 1e-14 * dt_o
    et = list(w.eos)
    _, gg, pi = tparams(w, True)
    m, mat = torch.as_tensor(w.m), torch.as_tensor(w.mat).long()
    st = {k: torch.as_tensor(s[k]).clone().requires_grad_(True) for k in F8}
    pairs = T.pairs_of(cfg, s)
    mir, wt = None, None
    if w.wall is not None:
        xw = w.wall[0] + w.wall[1] * t
        mir = T.mirror_pairs_of(s, H, xw, pair_h=ph)
        wt = (xw, w.wall[1])
    dtt = T.cfl_dt_torch(st, m, mat, et, gg, pi, pairs, H, 0.3, w.h, mirror=mir, wall=wt,
                         pair_h=ph)
    per = getattr(w, "periodic", 0)
    out = T.step_torch(st, m, mat, et, gg, pi, pairs, H, dtt, mirror=mir, wall=w.wall, t=t,
                       box=w.box, periodic=per, pair_h=ph)
    for k in F8:
        assert np.abs(out[k].detach().numpy() - base[k]).max() <= 1e-12 * (1 + np.abs(base[k]).max()), k
    J = sum((out[k] * torch.as_tensor(lam[k])).sum() for k in F8)
    ref = torch.autograd.grad(J, [st[k] for k in F8] + [gg, pi])
    for a, k in enumerate(F8):
        assert relmax(gp[k].cpu().numpy(), ref[a].numpy()) <= 1e-10, k
    ge = ge.cpu().numpy()
    assert relmax(ge[0::2], ref[8].numpy()) <= 1e-10
    if w.eos[-1][0] == 1:
        assert abs(ge[-1] - float(ref[9][-1])) <= 1e-10 * max(abs(float(ref[9][-1])), 1e-12)
    dd = {k: rng.standard_normal(w.n) for k in F8}
    eps = 1e-7
    (fp, _), (fm, _) = fwd(dd, eps), fwd(dd, -eps)
    jvp = sum(float(((fp[k] - fm[k]) / (2 * eps) * lam[k]).sum()) for k in F8)
    vjp = sum(float((gp[k].cpu().numpy() * dd[k]).sum()) for k in F8)
    assert abs(jvp - vjp) <= 1e-6 * max(abs(vjp), 1.0), (jvp, vjp)


def test_rollout_cfl_adjoint_fd_with_the_cfl_rule():
    """A rollout differentiated with its CFL steps (cfl_adjoint): central differences of the
    GPU rollout that reruns the CFL rule on every perturbed start agree with the gradient, and
    the FP64 CPU reference (autograd through dt) gives the same gradient; the frozen-dt
    gradient of the same run does not."""
    w = system(n=8, seed=47)
    params = P.Params.from_workload(w, cfl=0.3)
    base = _base(w, params)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64), device=DEV)
    v0 = [t(w.vx).requires_grad_(True), t(w.vy).requires_grad_(True), t(w.vz).requires_grad_(True)]
    gamma = torch.tensor([e[1] for e in w.eos], dtype=torch.float64, device=DEV,
                         requires_grad=True)
    nsteps, every = 8, 3
    info = {}
    out = P.rollout(*v0, gamma, base, params, nsteps, every, info=info, cfl_adjoint=True)
    mask = out["x"].detach() > 4.0
    J = _objective(out, mask, base["m"])
    grads = torch.autograd.grad(J, v0 + [gamma])
    out0 = P.rollout(*v0, gamma, base, params, nsteps, every, dts=info["dts"])
    g0 = torch.autograd.grad(_objective(out0, mask, base["m"]), v0 + [gamma])
    assert relmax(g0[3].cpu().numpy(), grads[3].cpu().numpy()) > 1e-3  # dt's part matters
    cfg = O.cfg_for(w)
    et, gg, pi = tparams(w, True)
    gg = gg.clone().detach().requires_grad_(True)
    mat = torch.as_tensor(w.mat).long()
    m = torch.as_tensor(w.m)
    vr = [torch.as_tensor(a).clone().requires_grad_(True) for a in (w.vx, w.vy, w.vz)]
    E0 = T.init_energy_torch(torch.as_tensor(w.rho), torch.as_tensor(w.p), *vr, mat, et, gg, pi)
    st = {"x": torch.as_tensor(w.x), "y": torch.as_tensor(w.y), "z": torch.as_tensor(w.z),
          "vx": vr[0], "vy": vr[1], "vz": vr[2], "rho": torch.as_tensor(w.rho), "E": E0}
    H = w.kappa * w.h
    for k in range(nsteps):
        pairs = T.pairs_of(cfg, {kk: st[kk].detach().numpy() for kk in ("x", "y", "z")})
        dtt = T.cfl_dt_torch(st, m, mat, et, gg, pi, pairs, H, 0.3, w.h)
        assert abs(float(dtt.detach()) - info["dts"][k]) <= 1e-13 * info["dts"][k]
        st = T.step_torch(st, m, mat, et, gg, pi, pairs, H, dtt)
    mref = st["x"].detach() > 4.0
    assert torch.equal(mref, mask.cpu())
    Jr = (st["vx"][mref] * m[mref]).sum()
    ref = torch.autograd.grad(Jr, vr + [gg])
    for a in range(3):
        assert relmax(grads[a].cpu().numpy(), ref[a].numpy()) <= 1e-9, a
    assert relmax(grads[3].cpu().numpy(), ref[3].numpy()) <= 1e-9
    rng = np.random.default_rng(48)
    for trial in range(4):
        dv = [rng.standard_normal(w.n) for _ in range(3)]
        dg = rng.standard_normal(len(w.eos))
        eps = 1e-7

        def Jat(sign):
            vv = [v0[a].detach() + sign * eps * t(dv[a]) for a in range(3)]
            gm = gamma.detach() + sign * eps * t(dg)
            o = P.rollout(*vv, gm, base, params, nsteps, every)  # the CFL rule, rerun
            return float(_objective(o, mask, base["m"]))

        fd = (Jat(1) - Jat(-1)) / (2 * eps)
        pred = sum(float((grads[a].cpu().numpy() * dv[a]).sum()) for a in range(3)) + \
            float((grads[3].cpu().numpy() * dg).sum())
        assert abs(fd - pred) <= 1e-4 * max(abs(pred), 1e-8), (trial, fd, pred)


def _rk2_case(name):
    """(workload, t, dt, extra Params fields, d or None)"""
    from test_adjoint_ref import periodic_system
    if name == "gas":
        return system(n=8, seed=61), 0.0, 0.08, {}, None
    if name == "piston":
        return piston_system(seed=62), 0.3, 0.2, {}, None
    if name == "periodic":
        return periodic_system(7, seed=63), 0.0, 0.2, {}, None
    w = system(n=8, seed=64)
    d = np.random.default_rng(64).uniform(0.8, 1.3, w.n)
    return w, 0.0, 0.08, dict(h_mode="pair", kappa=1.936, cell_size=0.0), d


@pytest.mark.parametrize("name", ["gas", "piston", "periodic", "pair-h"])
def test_rk2_step_vjp_matches_autograd_and_dot_product(name):
    """The RK2 step's VJP (two rate VJPs composed, dt fixed): against autograd of the FP64
    reference's RK2 step, and the dot-product test against the GPU's own RK2 steps."""
    w, t, dt, extra, d = _rk2_case(name)
    print(f"[case] rk2 vjp {name} n={w.n}", flush=True)
    params = P.Params.from_workload(w, reorder=False, integrator="rk2", **extra)
    replay = P.Params.from_workload(w, reorder=False, integrator="rk2", cfl=0.0, **extra)
    g = P.state_from_workload(w, params, DEV)
    if d is not None:
        g.d = torch.as_tensor(d, device=DEV)
    s = _np_state(g, w)
    H = w.kappa * w.h
    ph = None if d is None else (1.936, d)
    hm = dict(h_mode=1, kappa=1.936) if d is not None else {}
    cfg = O.cfg_for(w, **hm)
    per = getattr(w, "periodic", 0)
    box = getattr(w, "box", None)

    def fwd(delta=None, eps=0.0):
        tt = {k: g[k] + (eps * torch.as_tensor(delta[k], device=DEV) if delta else 0.0)
              for k in F8}
        tt["m"] = g["m"]
        st2 = P.State(tt, g.mat, g.d)
        P.csph_step(st2, replay, P.StepScalars(DEV, t0=t), s_out=st2, dt_in=dt)
        return {k: st2[k].cpu().numpy() for k in F8}

    base = fwd()
    rng = np.random.default_rng(110)
    lam = {k: rng.standard_normal(w.n) for k in F8}
    gn = {k: torch.as_tensor(v, device=DEV).clone() for k, v in lam.items()}
    gp, ge = P.csph_step_vjp(g, params, dt, gn, g_prev={k: torch.empty_like(v) for k, v in gn.items()},
                             t=t)

    def pairs_at(pos):
        q = dict(pos)
        if d is not None:
            q["d"] = d
        return T.pairs_of(cfg, q)

    def mirror_at(pos, xw):
        return T.mirror_pairs_of(pos, H, xw, box=box, periodic=per, pair_h=ph)

    et, gg, pi = tparams(w, True)
    m, mat = torch.as_tensor(w.m), torch.as_tensor(w.mat).long()
    st = {k: torch.as_tensor(s[k]).clone().requires_grad_(True) for k in F8}
    out = T.step_rk2_torch(st, m, mat, et, gg, pi, pairs_at, H, dt, mirror_at=mirror_at,
                           wall=w.wall, t=t, box=box, periodic=per, pair_h=ph)
    for k in F8:
        assert np.abs(out[k].detach().numpy() - base[k]).max() <= 1e-12 * (1 + np.abs(base[k]).max()), k
    J = sum((out[k] * torch.as_tensor(lam[k])).sum() for k in F8)
    ref = torch.autograd.grad(J, [st[k] for k in F8] + [gg, pi])
    for a, k in enumerate(F8):
        assert relmax(gp[k].cpu().numpy(), ref[a].numpy()) <= 1e-10, k
    assert relmax(ge.cpu().numpy()[0::2], ref[8].numpy()) <= 1e-10
    dd = {k: rng.standard_normal(w.n) for k in F8}
    eps = 1e-6
    fp, fm = fwd(dd, eps), fwd(dd, -eps)
    jvp = sum(float(((fp[k] - fm[k]) / (2 * eps) * lam[k]).sum()) for k in F8)
    vjp = sum(float((gp[k].cpu().numpy() * dd[k]).sum()) for k in F8)
    assert abs(jvp - vjp) <= 1e-7 * max(abs(vjp), 1.0), (jvp, vjp)


def test_rollout_rk2_piston_fd():
    """A rollout of RK2 steps with the piston (porous 10^3 sample, 8 FP64 CFL steps replayed,
    checkpoint every 3) against central differences of the GPU forward."""
    w = ci.config2(nside=10)
    params = P.Params.from_workload(w, cfl=0.3, integrator="rk2")
    base = _base(w, params)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64), device=DEV)
    v0 = [t(w.vx).requires_grad_(True), t(w.vy).requires_grad_(True), t(w.vz).requires_grad_(True)]
    gamma = torch.tensor([e[1] for e in w.eos], dtype=torch.float64, device=DEV,
                         requires_grad=True)
    nsteps, every, t0 = 8, 3, 0.05
    info = {}
    P.rollout(*v0, gamma, base, params, nsteps, every, info=info, t0=t0)
    dts = info["dts"]
    out = P.rollout(*v0, gamma, base, params, nsteps, every, dts=dts, t0=t0)
    mask = out["x"].detach() > float(np.median(w.x))
    J = _objective(out, mask, base["m"])
    grads = torch.autograd.grad(J, v0 + [gamma])
    rng = np.random.default_rng(111)
    for trial in range(4):
        dv = [rng.standard_normal(w.n) for _ in range(3)]
        dg = rng.standard_normal(len(w.eos))
        eps = 1e-6

        def Jat(sign):
            vv = [v0[a].detach() + sign * eps * t(dv[a]) for a in range(3)]
            gm = gamma.detach() + sign * eps * t(dg)
            o = P.rollout(*vv, gm, base, params, nsteps, every, dts=dts, t0=t0)
            return float(_objective(o, mask, base["m"]))

        fd = (Jat(1) - Jat(-1)) / (2 * eps)
        pred = sum(float((grads[a].cpu().numpy() * dv[a]).sum()) for a in range(3)) + \
            float((grads[3].cpu().numpy() * dg).sum())
        assert abs(fd - pred) <= 1e-4 * max(abs(pred), 1e-8), (trial, fd, pred)


def test_vjp_empty_and_lone_particle():
    """Edge cases: every VJP entry point on an empty state (nothing written, g_eos unchanged);
    the CFL step's VJP for one moving particle without partners, where s = c and dt =
    cfl h / c(e), e = E - |v|^2/2 (ideal gas: c^2 = gamma (gamma - 1) e), against the closed
    form of the gradient of J = lam . U' (U' = U except r' = r + dt v)."""
    params = P.Params(eos=[(0, 1.4, 0.0)])
    e0 = P.State.empty(0, DEV)
    z = {k: torch.zeros(0, dtype=torch.float64, device=DEV) for k in F8}
    ge = torch.zeros(2, dtype=torch.float64, device=DEV)
    cot = {k: torch.zeros(0, dtype=torch.float64, device=DEV) for k in ("drho", "dvx", "dvy", "dvz", "dE")}
    P.csph_rates_vjp(e0, params, cot, g_state=dict(z), g_eos=ge)
    P.csph_step_vjp(e0, params, 0.1, dict(z), g_eos=ge)
    P.csph_step_vjp(e0, P.Params(eos=[(0, 1.4, 0.0)], integrator="rk2"), 0.1, dict(z), g_eos=ge)
    P.csph_step_vjp_cfl(e0, params, dict(z), g_eos=ge)
    torch.cuda.synchronize()
    assert ge.abs().sum().item() == 0.0
    # one particle moving at v = (0.3, -0.2, 0.1)
    g, h, cfl = 1.4, 1.5, 0.3
    v = np.array([0.3, -0.2, 0.1])
    rho, p = 1.2, 0.8
    e = p / ((g - 1.0) * rho)
    E = e + 0.5 * float(v @ v)
    t1 = lambda a: torch.tensor([a], dtype=torch.float64, device=DEV)
    st = P.State({"x": t1(1.0), "y": t1(2.0), "z": t1(3.0), "vx": t1(v[0]), "vy": t1(v[1]),
                  "vz": t1(v[2]), "rho": t1(rho), "E": t1(E), "m": t1(rho)},
                 torch.zeros(1, dtype=torch.int32, device=DEV))
    prm = P.Params(eos=[(0, g, 0.0)], h=h, cfl=cfl, reorder=False)
    lam = {k: float(x) for k, x in zip(F8, np.random.default_rng(120).standard_normal(8))}
    gn = {k: t1(lam[k]) for k in F8}
    ge = torch.zeros(2, dtype=torch.float64, device=DEV)
    gp, ge, dt = P.csph_step_vjp_cfl(st, prm, gn, g_prev={k: t1(0.0) for k in F8}, g_eos=ge)
    c = np.sqrt(g * (g - 1.0) * e)
    assert abs(dt - cfl * h / c) <= 1e-15 * dt
    gdt = lam["x"] * v[0] + lam["y"] * v[1] + lam["z"] * v[2]   # dJ/d dt
    dtdc = -cfl * h / (c * c)
    dcde = g * (g - 1.0) / (2.0 * c)
    expect = {"x": lam["x"], "y": lam["y"], "z": lam["z"],
              "vx": lam["vx"] + dt * lam["x"] - gdt * dtdc * dcde * v[0],
              "vy": lam["vy"] + dt * lam["y"] - gdt * dtdc * dcde * v[1],
              "vz": lam["vz"] + dt * lam["z"] - gdt * dtdc * dcde * v[2],
              "rho": lam["rho"], "E": lam["E"] + gdt * dtdc * dcde}
    for k in F8:
        got = float(gp[k].item())
        assert abs(got - expect[k]) <= 1e-12 * max(1.0, abs(expect[k])), (k, got, expect[k])
    # d dt/d gamma through c^2 = gamma (gamma - 1) e
    dgamma = gdt * dtdc * (2.0 * g - 1.0) * e / (2.0 * c)
    assert abs(float(ge[0].item()) - dgamma) <= 1e-12 * max(1.0, abs(dgamma))


def test_step_vjp_lone_particle_reflected_by_the_piston():
    """A particle without partners (more than a support from the piston at t) that crosses
    it in one Euler step: the step reflects it, x'' = 2 x_w(t + dt) - (x + dt v_x),
    v_x'' = 2 v_w - v_x, E'' = E + (v_x''^2 - v_x^2)/2 (the rates vanish), and the VJP is the
    closed-form transpose of that map.  Also the empty state with the piston."""
    t, dt, xw0, vw = 0.2, 0.2, 0.0, 0.5
    prm = P.Params(eos=[(0, 1.4, 0.0)], h=1.5, cfl=0.0, reorder=False, wall=(xw0, vw))
    e0 = P.State.empty(0, DEV)
    z = {k: torch.zeros(0, dtype=torch.float64, device=DEV) for k in F8}
    cot = {k: torch.zeros(0, dtype=torch.float64, device=DEV) for k in ("drho", "dvx", "dvy", "dvz", "dE")}
    ge = torch.zeros(2, dtype=torch.float64, device=DEV)
    P.csph_rates_vjp(e0, prm, cot, g_state=dict(z), g_eos=ge, t=t)
    P.csph_step_vjp(e0, prm, dt, dict(z), g_eos=ge, t=t)
    torch.cuda.synchronize()
    assert ge.abs().sum().item() == 0.0
    v = np.array([-40.0, 0.3, -0.2])
    x0, rho, E = xw0 + vw * t + 6.0, 1.1, 2.5
    t1 = lambda a: torch.tensor([a], dtype=torch.float64, device=DEV)
    st = P.State({"x": t1(x0), "y": t1(2.0), "z": t1(3.0), "vx": t1(v[0]), "vy": t1(v[1]),
                  "vz": t1(v[2]), "rho": t1(rho), "E": t1(E), "m": t1(rho)},
                 torch.zeros(1, dtype=torch.int32, device=DEV))
    out = P.State.empty(1, DEV, True, False, False)
    P.csph_step(st, prm, P.StepScalars(DEV, t0=t), s_out=out, dt_in=dt, totals=False)
    xw1 = xw0 + vw * (t + dt)
    vx2 = 2.0 * vw - v[0]
    want = {"x": 2.0 * xw1 - (x0 + dt * v[0]), "y": 2.0 + dt * v[1], "z": 3.0 + dt * v[2],
            "vx": vx2, "vy": v[1], "vz": v[2], "rho": rho,
            "E": E + 0.5 * (vx2 * vx2 - v[0] * v[0])}
    for k in F8:
        assert abs(float(out[k].item()) - want[k]) <= 1e-13 * max(1.0, abs(want[k])), k
    lam = {k: float(x) for k, x in zip(F8, np.random.default_rng(121).standard_normal(8))}
    gn = {k: t1(lam[k]) for k in F8}
    gp, ge = P.csph_step_vjp(st, prm, dt, gn, g_prev={k: t1(0.0) for k in F8},
                             g_eos=torch.zeros(2, dtype=torch.float64, device=DEV), t=t)
    expect = {"x": -lam["x"], "y": lam["y"], "z": lam["z"],
              "vx": -dt * lam["x"] - lam["vx"] - 2.0 * vw * lam["E"],
              "vy": lam["vy"] + dt * lam["y"], "vz": lam["vz"] + dt * lam["z"],
              "rho": lam["rho"], "E": lam["E"]}
    for k in F8:
        got = float(gp[k].item())
        assert abs(got - expect[k]) <= 1e-13 * max(1.0, abs(expect[k])), (k, got, expect[k])
    assert float(ge.abs().sum().item()) == 0.0


def test_rk2_step_vjp_grows_a_fresh_workspace():
    """The RK2 step's VJP on a fresh, small workspace: it learns its scratch and both meshes'
    needs over the binding's retries and returns the same gradient as with a large one."""
    w, t, dt, extra, d = _rk2_case("piston")
    params = P.Params.from_workload(w, reorder=False, integrator="rk2", **extra)
    g = P.state_from_workload(w, params, DEV)
    rng = np.random.default_rng(130)
    gn = {k: torch.as_tensor(rng.standard_normal(w.n), device=DEV) for k in F8}
    big = P.Workspace(DEV)
    big.ensure(1 << 28)
    ga, ea = P.csph_step_vjp(g, params, dt, gn, g_prev={k: torch.empty_like(v) for k, v in gn.items()},
                             ws=big, t=t)
    small = P.Workspace(DEV)
    gb, eb = P.csph_step_vjp(g, params, dt, gn, g_prev={k: torch.empty_like(v) for k, v in gn.items()},
                             ws=small, t=t)
    torch.cuda.synchronize()
    for k in F8:
        assert torch.equal(ga[k], gb[k]), k
    assert torch.equal(ea, eb)


@pytest.mark.parametrize("kind", ["euler", "cfl", "rk2"])
def test_step_vjp_with_the_piston_in_place(kind):
    """The step VJPs with the piston write g_prev over g_next (the rollout's in-place use)
    with the same result, bit for bit, as into separate arrays."""
    w = piston_system(seed=7)
    t, dt = 0.3, 0.2
    params = P.Params.from_workload(w, reorder=False, cfl=0.3 if kind == "cfl" else 0.0,
                                    integrator="rk2" if kind == "rk2" else "euler")
    g = P.state_from_workload(w, params, DEV)
    rng = np.random.default_rng(140)
    lam = {k: torch.as_tensor(rng.standard_normal(w.n), device=DEV) for k in F8}

    def run(inplace):
        gn = {k: v.clone() for k, v in lam.items()}
        gp = gn if inplace else {k: torch.empty_like(v) for k, v in gn.items()}
        if kind == "cfl":
            out, ge, _ = P.csph_step_vjp_cfl(g, params, gn, g_prev=gp, t=t)
        else:
            out, ge = P.csph_step_vjp(g, params, dt, gn, g_prev=gp, t=t)
        torch.cuda.synchronize()
        return out, ge

    a, ea = run(False)
    b, eb = run(True)
    for k in F8:
        assert torch.equal(a[k], b[k]), k
    assert torch.equal(ea, eb)
