"""Pins of the differentiable CPU reference (oracle/torch_ref.py).

Its forward must reproduce the C oracle; its autograd gradients must match
central finite differences of the C oracle's own step (an independent code
path), along random directions in state and EOS-parameter space.
"""
import numpy as np
import pytest
import torch

import csph_inputs as ci
import oracle as O
from oracle import torch_ref as T

F8 = T.FIELDS8


def system(n=6, seed=3, two_mat=True):
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


def tparams(w):
    gamma = torch.tensor([e[1] for e in w.eos], dtype=torch.float64)
    pinf = torch.tensor([e[2] for e in w.eos], dtype=torch.float64)
    return [e[0] for e in w.eos], gamma, pinf


def test_torch_rates_match_c_oracle():
    w = system()
    cfg = O.cfg_for(w)
    s = O.state_from(w, cfg)
    ref = O.rates(cfg, s)
    et, g, pi = tparams(w)
    out = T.rates_torch(T.to_torch(s), torch.as_tensor(s["m"]), torch.as_tensor(s["mat"]).long(),
                        et, g, pi, T.pairs_of(cfg, s), w.kappa * w.h)
    for k, v in zip(("drho", "dvx", "dvy", "dvz", "dE"), out):
        scale = np.abs(ref[k]).max()
        assert np.abs(v.numpy() - ref[k]).max() <= 1e-13 * scale, k


def _oracle_step(w, s, eos, dt):
    cfg = O.make_cfg(eos, h=w.h, kappa=w.kappa, cfl=0.0)
    s1, _, _, _ = O.step(cfg, s, 0.0, dt_in=dt)
    return s1


@pytest.mark.parametrize("seed", [3, 4])
def test_step_gradient_matches_oracle_finite_differences(seed):
    w = system(seed=seed)
    cfg = O.cfg_for(w)
    s = O.state_from(w, cfg)
    dt = 0.05
    et, g, pi = tparams(w)
    st = {k: v.clone().requires_grad_(True) for k, v in T.to_torch(s).items()}
    g = g.clone().requires_grad_(True)
    pi = pi.clone().requires_grad_(True)
    m = torch.as_tensor(s["m"])
    mat = torch.as_tensor(s["mat"]).long()
    out = T.step_torch(st, m, mat, et, g, pi, T.pairs_of(cfg, s), w.kappa * w.h, dt)
    rng = np.random.default_rng(seed + 10)
    lam = {k: rng.standard_normal(w.n) for k in F8}
    J = sum((out[k] * torch.as_tensor(lam[k])).sum() for k in F8)
    grads = torch.autograd.grad(J, [st[k] for k in F8] + [g, pi])
    for trial in range(3):
        d = {k: rng.standard_normal(w.n) for k in F8}
        dg = rng.standard_normal(len(w.eos))
        dpi = rng.standard_normal(len(w.eos)) * np.array([0.0 if e[0] == 0 else 1.0 for e in w.eos])
        pred = sum(float((grads[a].numpy() * d[k]).sum()) for a, k in enumerate(F8))
        pred += float((grads[8].numpy() * dg).sum()) + float((grads[9].numpy() * dpi).sum())
        eps = 1e-6

        def J_at(sign):
            s2 = {k: (s[k] + sign * eps * d[k]) if k in d else s[k] for k in s}
            eos2 = [(e[0], e[1] + sign * eps * dg[k], e[2] + sign * eps * dpi[k])
                    for k, e in enumerate(w.eos)]
            s1 = _oracle_step(w, s2, eos2, dt)
            return sum(float((s1[k] * lam[k]).sum()) for k in F8)

        fd = (J_at(1) - J_at(-1)) / (2 * eps)
        assert abs(fd - pred) <= 1e-6 * max(abs(pred), 1.0), (trial, fd, pred)


def test_init_energy_gamma_gradient():
    w = system(two_mat=True)
    et, g, pi = tparams(w)
    g = g.clone().requires_grad_(True)
    pi = pi.clone().requires_grad_(True)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64))
    mat = torch.as_tensor(w.mat).long()
    E = T.init_energy_torch(t(w.rho), t(w.p), t(w.vx), t(w.vy), t(w.vz), mat, et, g, pi)
    lam = np.random.default_rng(0).standard_normal(w.n)
    J = (E * t(lam)).sum()
    gg, gp = torch.autograd.grad(J, [g, pi])
    eps = 1e-7
    for k in range(len(w.eos)):
        for which, grad in ((1, gg), (2, gp)):
            if which == 2 and w.eos[k][0] == 0:
                continue

            def Jat(sign):
                eos2 = [list(e) for e in w.eos]
                eos2[k][which] += sign * eps
                cfg = O.make_cfg([tuple(e) for e in eos2])
                E2 = O.init_energy(cfg, w.rho, w.p, w.vx, w.vy, w.vz, w.mat)
                return float((E2 * lam).sum())

            fd = (Jat(1) - Jat(-1)) / (2 * eps)
            assert abs(fd - float(grad[k])) <= 1e-6 * max(1.0, abs(fd))


def wall_system(seed=5):
    """The block moving onto the piston (x_w = 0.2 + 0.4 t): at t = 0.3 the first layers have
    mirror partners, and a step of 0.2 reflects about half of the first layer."""
    w = system(n=6, seed=seed)
    w.vx = w.vx - 0.5
    w.wall = (0.2, 0.4)
    return w


def test_torch_rates_with_the_piston_match_c_oracle():
    w = wall_system()
    cfg = O.cfg_for(w)
    s = O.state_from(w, cfg)
    t = 0.3
    ref = O.rates(cfg, s, t=t)
    et, g, pi = tparams(w)
    xw = w.wall[0] + w.wall[1] * t
    mir = T.mirror_pairs_of(s, w.kappa * w.h, xw)
    assert len(mir[0]) > 20
    out = T.rates_torch(T.to_torch(s), torch.as_tensor(s["m"]), torch.as_tensor(s["mat"]).long(),
                        et, g, pi, T.pairs_of(cfg, s), w.kappa * w.h, mirror=mir,
                        wall=(xw, w.wall[1]))
    for k, v in zip(("drho", "dvx", "dvy", "dvz", "dE"), out):
        scale = np.abs(ref[k]).max()
        assert np.abs(v.numpy() - ref[k]).max() <= 1e-13 * scale, k


@pytest.mark.parametrize("seed", [5, 6])
def test_step_with_the_piston_gradient_matches_oracle_finite_differences(seed):
    """Mirror partners and reflections in the step: the reference's gradient (reflection
    branches and mirror pairs fixed at the base state) against central differences of the
    C oracle's step with the piston."""
    w = wall_system(seed)
    cfg = O.cfg_for(w, cfl=0.0)  # the step takes dt_in as given
    s = O.state_from(w, cfg)
    t, dt = 0.3, 0.2
    s1_base, _, _, _ = O.step(cfg, s, t, dt_in=dt)
    assert np.sum(s1_base["vx"] > 0.3) > 3  # some particles were reflected
    et, g, pi = tparams(w)
    st = {k: v.clone().requires_grad_(True) for k, v in T.to_torch(s).items()}
    g = g.clone().requires_grad_(True)
    pi = pi.clone().requires_grad_(True)
    m = torch.as_tensor(s["m"])
    mat = torch.as_tensor(s["mat"]).long()
    mir = T.mirror_pairs_of(s, w.kappa * w.h, w.wall[0] + w.wall[1] * t)
    out = T.step_torch(st, m, mat, et, g, pi, T.pairs_of(cfg, s), w.kappa * w.h, dt,
                       mirror=mir, wall=w.wall, t=t)
    for k in F8:
        assert np.abs(out[k].detach().numpy() - s1_base[k]).max() <= 1e-13 * (1 + np.abs(s1_base[k]).max()), k
    rng = np.random.default_rng(seed + 20)
    lam = {k: rng.standard_normal(w.n) for k in F8}
    J = sum((out[k] * torch.as_tensor(lam[k])).sum() for k in F8)
    grads = torch.autograd.grad(J, [st[k] for k in F8] + [g, pi])
    for trial in range(3):
        d = {k: rng.standard_normal(w.n) for k in F8}
        dg = rng.standard_normal(len(w.eos))
        dpi = rng.standard_normal(len(w.eos)) * np.array([0.0 if e[0] == 0 else 1.0 for e in w.eos])
        pred = sum(float((grads[a].numpy() * d[k]).sum()) for a, k in enumerate(F8))
        pred += float((grads[8].numpy() * dg).sum()) + float((grads[9].numpy() * dpi).sum())
        eps = 1e-6

        def J_at(sign):
            s2 = {k: (s[k] + sign * eps * d[k]) if k in d else s[k] for k in s}
            eos2 = [(e[0], e[1] + sign * eps * dg[k], e[2] + sign * eps * dpi[k])
                    for k, e in enumerate(w.eos)]
            c2 = O.make_cfg(eos2, h=w.h, kappa=w.kappa, cfl=0.0, wall=w.wall)
            s1, _, _, _ = O.step(c2, s2, t, dt_in=dt)
            return sum(float((s1[k] * lam[k]).sum()) for k in F8)

        fd = (J_at(1) - J_at(-1)) / (2 * eps)
        assert abs(fd - pred) <= 1e-6 * max(abs(pred), 1.0), (trial, fd, pred)


def mg_system(n=6, seed=7):
    """An ideal gas and a Mie-Grueneisen solid (aluminium-like constants) side by side, the
    solid compressed by 0-8 % or expanded by up to 3 % against rho0."""
    w = system(n=n, seed=seed)
    rng = np.random.default_rng(seed + 1)
    solid = w.mat == 1
    w.rho = np.where(solid, ci.MG_ALUMINIUM[3] * rng.uniform(0.97, 1.08, w.n), w.rho)
    w.m = w.rho.copy()
    w.eos = [(0, 1.4, 0.0), ci.MG_ALUMINIUM]
    return w


def _eos_shifted(eos, sign, eps, dg, dpi):
    """The materials with gamma (Gamma) and p_inf moved along (dg, dpi); other constants kept."""
    return [(e[0], e[1] + sign * eps * dg[k], e[2] + sign * eps * dpi[k]) + tuple(e[3:])
            for k, e in enumerate(eos)]


def test_torch_rates_with_mie_grueneisen_match_c_oracle():
    w = mg_system()
    cfg = O.cfg_for(w)
    s = O.state_from(w, cfg)
    P, c, bad = O.eos(cfg, s)
    assert bad == 0 and np.all(c > 0.0)
    ref = O.rates(cfg, s)
    _, g, pi = tparams(w)
    st = T.to_torch(s)
    mat = torch.as_tensor(s["mat"]).long()
    Pt, ct = T.eos_torch(st["rho"], st["E"], st["vx"], st["vy"], st["vz"], mat, list(w.eos), g,
                         pi)
    assert np.abs(Pt.numpy() - P).max() <= 1e-13 * np.abs(P).max()
    assert np.abs(ct.numpy() - c).max() <= 1e-13 * np.abs(c).max()
    out = T.rates_torch(st, torch.as_tensor(s["m"]), mat, list(w.eos), g, pi, T.pairs_of(cfg, s),
                        w.kappa * w.h)
    for k, v in zip(("drho", "dvx", "dvy", "dvz", "dE"), out):
        scale = np.abs(ref[k]).max()
        assert np.abs(v.numpy() - ref[k]).max() <= 1e-12 * scale, k


@pytest.mark.parametrize("seed", [7, 8])
def test_step_with_mie_grueneisen_gradient_matches_oracle_finite_differences(seed):
    """Gradients through the Mie-Grueneisen pressure and sound speed (and Gamma) against
    central differences of the C oracle's step."""
    w = mg_system(seed=seed)
    cfg = O.cfg_for(w, cfl=0.0)
    s = O.state_from(w, cfg)
    dt = 0.02
    _, g, pi = tparams(w)
    st = {k: v.clone().requires_grad_(True) for k, v in T.to_torch(s).items()}
    g = g.clone().requires_grad_(True)
    pi = pi.clone().requires_grad_(True)
    m = torch.as_tensor(s["m"])
    mat = torch.as_tensor(s["mat"]).long()
    out = T.step_torch(st, m, mat, list(w.eos), g, pi, T.pairs_of(cfg, s), w.kappa * w.h, dt)
    rng = np.random.default_rng(seed + 40)
    lam = {k: rng.standard_normal(w.n) for k in F8}
    J = sum((out[k] * torch.as_tensor(lam[k])).sum() for k in F8)
    grads = torch.autograd.grad(J, [st[k] for k in F8] + [g, pi])
    assert float(grads[9][1]) == 0.0  # the solid has no p_inf
    for trial in range(3):
        d = {k: rng.standard_normal(w.n) for k in F8}
        dg = rng.standard_normal(len(w.eos))
        dpi = np.zeros(len(w.eos))
        pred = sum(float((grads[a].numpy() * d[k]).sum()) for a, k in enumerate(F8))
        pred += float((grads[8].numpy() * dg).sum())
        eps = 1e-6

        def J_at(sign):
            s2 = {k: (s[k] + sign * eps * d[k]) if k in d else s[k] for k in s}
            c2 = O.make_cfg(_eos_shifted(w.eos, sign, eps, dg, dpi), h=w.h, kappa=w.kappa,
                            cfl=0.0)
            s1, _, _, _ = O.step(c2, s2, 0.0, dt_in=dt)
            return sum(float((s1[k] * lam[k]).sum()) for k in F8)

        fd = (J_at(1) - J_at(-1)) / (2 * eps)
        assert abs(fd - pred) <= 1e-6 * max(abs(pred), 1.0), (trial, fd, pred)


def test_init_energy_with_mie_grueneisen_matches_oracle():
    """E0 of the solid from (rho, p): value against the C oracle, and d/d(rho, Gamma) against
    central differences of it."""
    w = mg_system(seed=9)
    cfg = O.cfg_for(w)
    E_ref = O.init_energy(cfg, w.rho, w.p, w.vx, w.vy, w.vz, w.mat)
    _, g, pi = tparams(w)
    g = g.clone().requires_grad_(True)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64))
    rho = t(w.rho).clone().requires_grad_(True)
    mat = torch.as_tensor(w.mat).long()
    E = T.init_energy_torch(rho, t(w.p), t(w.vx), t(w.vy), t(w.vz), mat, list(w.eos), g, pi)
    assert np.abs(E.detach().numpy() - E_ref).max() <= 1e-13 * np.abs(E_ref).max()
    lam = np.random.default_rng(3).standard_normal(w.n)
    grho, gg = torch.autograd.grad((E * t(lam)).sum(), [rho, g])
    eps = 1e-7
    dr = np.random.default_rng(4).standard_normal(w.n)
    for k in range(len(w.eos)):
        def Jg(sign):
            eos2 = [list(e) for e in w.eos]
            eos2[k][1] += sign * eps
            E2 = O.init_energy(O.make_cfg([tuple(e) for e in eos2]), w.rho, w.p, w.vx, w.vy,
                               w.vz, w.mat)
            return float((E2 * lam).sum())

        fd = (Jg(1) - Jg(-1)) / (2 * eps)
        assert abs(fd - float(gg[k])) <= 1e-6 * max(1.0, abs(fd)), k

    def Jr(sign):
        E2 = O.init_energy(cfg, w.rho + sign * eps * dr, w.p, w.vx, w.vy, w.vz, w.mat)
        return float((E2 * lam).sum())

    fd = (Jr(1) - Jr(-1)) / (2 * eps)
    pred = float((grho.numpy() * dr).sum())
    assert abs(fd - pred) <= 1e-6 * max(1.0, abs(pred))


def periodic_system(periodic=7, seed=11, wall=None):
    """A 7 x 8 x 7 jittered lattice filling its box, periodic along ``periodic``; two gases,
    velocities of 1-2 so that particles leave through the faces in a step."""
    w = ci.periodic_block(7, 8, 7, seed=seed, periodic=periodic, amp=0.3)
    rng = np.random.default_rng(seed)
    w.vx, w.vy, w.vz = (rng.uniform(-0.5, 0.5, w.n) for _ in range(3))
    w.vy = w.vy + 1.5
    w.vz = w.vz - 1.2
    w.rho = rng.uniform(0.8, 1.3, w.n)
    w.p = rng.uniform(0.5, 1.5, w.n)
    w.m = w.rho.copy()
    w.mat = (w.z > 3.5).astype(np.int32)
    w.eos = [(0, 1.4, 0.0), (1, 3.0, 0.4)]
    if wall is not None:
        w.vx = w.vx - 0.5
        w.wall = wall
    return w


@pytest.mark.parametrize("periodic,wall", [(7, None), (5, None), (6, (0.2, 0.4))],
                         ids=["xyz", "xz", "yz+piston"])
def test_torch_rates_periodic_match_c_oracle(periodic, wall):
    w = periodic_system(periodic, wall=wall)
    cfg = O.cfg_for(w)
    s = O.state_from(w, cfg)
    t = 0.3
    ref = O.rates(cfg, s, t=t)
    et, g, pi = tparams(w)
    pairs = T.pairs_of(cfg, s)
    assert float(pairs[2].abs().max()) > 0.0  # image partners present
    mir, wt = None, None
    if wall is not None:
        xw = wall[0] + wall[1] * t
        mir = T.mirror_pairs_of(s, w.kappa * w.h, xw, box=w.box, periodic=periodic)
        assert float(mir[2].abs().max()) > 0.0  # mirror partners through the images
        wt = (xw, wall[1])
    out = T.rates_torch(T.to_torch(s), torch.as_tensor(s["m"]), torch.as_tensor(s["mat"]).long(),
                        et, g, pi, pairs, w.kappa * w.h, mirror=mir, wall=wt)
    for k, v in zip(("drho", "dvx", "dvy", "dvz", "dE"), out):
        scale = np.abs(ref[k]).max()
        assert np.abs(v.numpy() - ref[k]).max() <= 1e-13 * scale, k


@pytest.mark.parametrize("periodic,wall", [(7, None), (6, (0.2, 0.4))], ids=["xyz", "yz+piston"])
def test_step_periodic_gradient_matches_oracle_finite_differences(periodic, wall):
    """Image partners, the wrap into the box (a translation) and, with the piston on periodic
    sides, mirror partners through the images: the reference's gradient against central
    differences of the C oracle's step."""
    w = periodic_system(periodic, seed=12, wall=wall)
    cfg = O.cfg_for(w, cfl=0.0)
    s = O.state_from(w, cfg)
    t, dt = 0.3, 0.2
    s1_base, _, _, _ = O.step(cfg, s, t, dt_in=dt)
    wrapped = np.abs(s1_base["y"] - s["y"]) > 4.0
    assert wrapped.sum() > 3  # particles left through a face and re-entered
    et, g, pi = tparams(w)
    st = {k: v.clone().requires_grad_(True) for k, v in T.to_torch(s).items()}
    g = g.clone().requires_grad_(True)
    pi = pi.clone().requires_grad_(True)
    m = torch.as_tensor(s["m"])
    mat = torch.as_tensor(s["mat"]).long()
    mir = None
    if wall is not None:
        mir = T.mirror_pairs_of(s, w.kappa * w.h, wall[0] + wall[1] * t, box=w.box,
                                periodic=periodic)
    out = T.step_torch(st, m, mat, et, g, pi, T.pairs_of(cfg, s), w.kappa * w.h, dt,
                       mirror=mir, wall=wall, t=t, box=w.box, periodic=periodic)
    for k in F8:
        assert np.abs(out[k].detach().numpy() - s1_base[k]).max() <= 1e-13 * (1 + np.abs(s1_base[k]).max()), k
    rng = np.random.default_rng(50)
    lam = {k: rng.standard_normal(w.n) for k in F8}
    J = sum((out[k] * torch.as_tensor(lam[k])).sum() for k in F8)
    grads = torch.autograd.grad(J, [st[k] for k in F8] + [g, pi])
    for trial in range(3):
        d = {k: rng.standard_normal(w.n) for k in F8}
        dg = rng.standard_normal(len(w.eos))
        dpi = rng.standard_normal(len(w.eos)) * np.array([0.0 if e[0] == 0 else 1.0 for e in w.eos])
        pred = sum(float((grads[a].numpy() * d[k]).sum()) for a, k in enumerate(F8))
        pred += float((grads[8].numpy() * dg).sum()) + float((grads[9].numpy() * dpi).sum())
        eps = 1e-6

        def J_at(sign):
            s2 = {k: (s[k] + sign * eps * d[k]) if k in d else s[k] for k in s}
            c2 = O.make_cfg(_eos_shifted(w.eos, sign, eps, dg, dpi), h=w.h, kappa=w.kappa,
                            cfl=0.0, wall=wall, periodic=periodic, box=w.box)
            s1, _, _, _ = O.step(c2, s2, t, dt_in=dt)
            return sum(float((s1[k] * lam[k]).sum()) for k in F8)

        fd = (J_at(1) - J_at(-1)) / (2 * eps)
        assert abs(fd - pred) <= 1e-6 * max(abs(pred), 1.0), (trial, fd, pred)


def pair_h_system(seed=21, wall=None):
    """Pair-h mode (support kappa (d_i + d_j)/2, kappa = 1.936) with particle sizes 0.8-1.3."""
    w = system(n=6, seed=seed)
    rng = np.random.default_rng(seed + 3)
    d = rng.uniform(0.8, 1.3, w.n)
    if wall is not None:
        w.vx = w.vx - 0.5
        w.wall = wall
    return w, d


@pytest.mark.parametrize("wall", [None, (0.2, 0.4)], ids=["open", "piston"])
def test_torch_rates_pair_h_match_c_oracle(wall):
    w, d = pair_h_system(wall=wall)
    cfg = O.cfg_for(w, h_mode=1, kappa=1.936)
    s = O.state_from(w, cfg)
    s["d"] = d
    t = 0.3
    ref = O.rates(cfg, s, t=t, d=d)
    et, g, pi = tparams(w)
    ph = (1.936, d)
    mir, wt = None, None
    if wall is not None:
        xw = wall[0] + wall[1] * t
        mir = T.mirror_pairs_of(s, 0.0, xw, pair_h=ph)
        assert len(mir[0]) > 10
        wt = (xw, wall[1])
    out = T.rates_torch(T.to_torch(s), torch.as_tensor(s["m"]), torch.as_tensor(s["mat"]).long(),
                        et, g, pi, T.pairs_of(cfg, s), 0.0, mirror=mir, wall=wt, pair_h=ph)
    for k, v in zip(("drho", "dvx", "dvy", "dvz", "dE"), out):
        scale = np.abs(ref[k]).max()
        assert np.abs(v.numpy() - ref[k]).max() <= 1e-13 * scale, k


@pytest.mark.parametrize("wall", [None, (0.2, 0.4)], ids=["open", "piston"])
def test_step_pair_h_gradient_matches_oracle_finite_differences(wall):
    """Pair-h mode (each pair's own support, d held fixed): the reference's gradient against
    central differences of the C oracle's step."""
    w, d = pair_h_system(seed=22, wall=wall)
    cfg = O.cfg_for(w, h_mode=1, kappa=1.936, cfl=0.0)
    s = O.state_from(w, cfg)
    s["d"] = d
    t, dt = 0.3, 0.1
    ph = (1.936, d)
    et, g, pi = tparams(w)
    st = {k: v.clone().requires_grad_(True) for k, v in T.to_torch(s).items()}
    g = g.clone().requires_grad_(True)
    pi = pi.clone().requires_grad_(True)
    m = torch.as_tensor(s["m"])
    mat = torch.as_tensor(s["mat"]).long()
    mir = None if wall is None else T.mirror_pairs_of(s, 0.0, wall[0] + wall[1] * t, pair_h=ph)
    out = T.step_torch(st, m, mat, et, g, pi, T.pairs_of(cfg, s), 0.0, dt, mirror=mir,
                       wall=wall, t=t, pair_h=ph)
    s1_base, _, _, _ = O.step(cfg, s, t, dt_in=dt, d=d)
    for k in F8:
        assert np.abs(out[k].detach().numpy() - s1_base[k]).max() <= 1e-13 * (1 + np.abs(s1_base[k]).max()), k
    rng = np.random.default_rng(70)
    lam = {k: rng.standard_normal(w.n) for k in F8}
    J = sum((out[k] * torch.as_tensor(lam[k])).sum() for k in F8)
    grads = torch.autograd.grad(J, [st[k] for k in F8] + [g, pi])
    for trial in range(3):
        dd = {k: rng.standard_normal(w.n) for k in F8}
        dg = rng.standard_normal(len(w.eos))
        dpi = rng.standard_normal(len(w.eos)) * np.array([0.0 if e[0] == 0 else 1.0 for e in w.eos])
        pred = sum(float((grads[a].numpy() * dd[k]).sum()) for a, k in enumerate(F8))
        pred += float((grads[8].numpy() * dg).sum()) + float((grads[9].numpy() * dpi).sum())
        eps = 1e-6

        def J_at(sign):
            s2 = {k: (s[k] + sign * eps * dd[k]) if k in dd else s[k] for k in s}
            c2 = O.make_cfg(_eos_shifted(w.eos, sign, eps, dg, dpi), h=w.h, kappa=1.936,
                            h_mode=1, cfl=0.0, wall=wall)
            s1, _, _, _ = O.step(c2, s2, t, dt_in=dt, d=d)
            return sum(float((s1[k] * lam[k]).sum()) for k in F8)

        fd = (J_at(1) - J_at(-1)) / (2 * eps)
        assert abs(fd - pred) <= 1e-6 * max(abs(pred), 1.0), (trial, fd, pred)


def expanding_system(seed=34):
    """A gas cube expanding from its centre (v = 2 (r - r_c)): the density-change limit sets
    the time step, not the Courant limit."""
    w = system(n=6, seed=seed)
    for k in ("x", "y", "z"):
        v = getattr(w, k)
        setattr(w, "v" + k, 2.0 * (v - v.mean()))
    return w


@pytest.mark.parametrize("case", ["gas", "piston", "mg", "expanding"])
def test_cfl_step_gradient_matches_oracle_finite_differences(case):
    """The CFL time step differentiated with the step: dt = cfl min_i min(h / s_i,
    rho_i / |drho_i|) from the reference (the minimum and the signal speed's maxima pass
    their gradients to the particle and partner that attain them) against central
    differences of the C oracle's step, which recomputes dt on every perturbed state."""
    w = {"gas": lambda: system(n=6, seed=31), "piston": lambda: wall_system(seed=32),
         "mg": lambda: mg_system(seed=33), "expanding": expanding_system}[case]()
    cfg = O.cfg_for(w, cfl=0.3)
    s = O.state_from(w, cfg)
    t = 0.3 if w.wall is not None else 0.0
    et = list(w.eos)
    _, g, pi = tparams(w)
    st = {k: v.clone().requires_grad_(True) for k, v in T.to_torch(s).items()}
    g = g.clone().requires_grad_(True)
    pi = pi.clone().requires_grad_(True)
    m = torch.as_tensor(s["m"])
    mat = torch.as_tensor(s["mat"]).long()
    H = w.kappa * w.h
    pairs = T.pairs_of(cfg, s)
    mir, wt = None, None
    if w.wall is not None:
        xw = w.wall[0] + w.wall[1] * t
        mir = T.mirror_pairs_of(s, H, xw)
        wt = (xw, w.wall[1])
    dt = T.cfl_dt_torch(st, m, mat, et, g, pi, pairs, H, 0.3, w.h, mirror=mir, wall=wt)
    s1_base, _, dt_o, _ = O.step(cfg, s, t)
    assert abs(float(dt.detach()) - dt_o) <= 1e-14 * dt_o
    out = T.step_torch(st, m, mat, et, g, pi, pairs, H, dt, mirror=mir, wall=w.wall, t=t)
    for k in F8:
        assert np.abs(out[k].detach().numpy() - s1_base[k]).max() <= 1e-13 * (1 + np.abs(s1_base[k]).max()), k
    rng = np.random.default_rng(80)
    lam = {k: rng.standard_normal(w.n) for k in F8}
    J = sum((out[k] * torch.as_tensor(lam[k])).sum() for k in F8)
    grads = torch.autograd.grad(J, [st[k] for k in F8] + [g, pi])
    # the dt term is not small: the frozen-dt gradient differs
    st0 = {k: v.detach().clone().requires_grad_(True) for k, v in T.to_torch(s).items()}
    out0 = T.step_torch(st0, m, mat, et, g.detach(), pi.detach(), pairs, H, float(dt.detach()),
                        mirror=mir, wall=w.wall, t=t)
    J0 = sum((out0[k] * torch.as_tensor(lam[k])).sum() for k in F8)
    g0 = torch.autograd.grad(J0, [st0[k] for k in F8])
    assert max(float((g0[a] - grads[a]).abs().max()) for a in range(8)) > 1e-3
    for trial in range(3):
        d = {k: rng.standard_normal(w.n) for k in F8}
        dg = rng.standard_normal(len(w.eos))
        dpi = np.zeros(len(w.eos))
        pred = sum(float((grads[a].numpy() * d[k]).sum()) for a, k in enumerate(F8))
        pred += float((grads[8].numpy() * dg).sum())
        eps = 1e-7

        def J_at(sign):
            s2 = {k: (s[k] + sign * eps * d[k]) if k in d else s[k] for k in s}
            c2 = O.make_cfg(_eos_shifted(w.eos, sign, eps, dg, dpi), h=w.h, kappa=w.kappa,
                            cfl=0.3, wall=w.wall)
            s1, _, _, _ = O.step(c2, s2, t)
            return sum(float((s1[k] * lam[k]).sum()) for k in F8)

        fd = (J_at(1) - J_at(-1)) / (2 * eps)
        assert abs(fd - pred) <= 1e-6 * max(abs(pred), 1.0), (trial, fd, pred)


@pytest.mark.parametrize("case", ["gas", "piston", "periodic", "pair-h"])
def test_rk2_step_gradient_matches_oracle_finite_differences(case):
    """The two-stage Runge-Kutta step (second evaluation at U1 and t + dt, wrapped positions,
    the piston's mirror partners there): the reference's forward against the C oracle's RK2
    step and its gradient against central differences of it."""
    d, ph, hm = None, None, {}
    if case == "gas":
        w, t, dt = system(n=6, seed=51), 0.0, 0.1
    elif case == "piston":
        w, t, dt = wall_system(seed=52), 0.3, 0.2
    elif case == "periodic":
        w, t, dt = periodic_system(7, seed=53), 0.0, 0.2
    else:
        w, d = pair_h_system(seed=54)
        t, dt, ph, hm = 0.0, 0.1, (1.936, d), dict(h_mode=1, kappa=1.936)
    cfg = O.cfg_for(w, cfl=0.0, integrator=1, **hm)
    s = O.state_from(w, cfg)
    if d is not None:
        s["d"] = d
    H = w.kappa * w.h
    per = getattr(w, "periodic", 0)
    box = getattr(w, "box", None)

    def pairs_at(pos):
        q = dict(pos)
        if d is not None:
            q["d"] = d
        return T.pairs_of(cfg, q)

    def mirror_at(pos, xw):
        return T.mirror_pairs_of(pos, H, xw, box=box, periodic=per, pair_h=ph)

    et, g, pi = tparams(w)
    st = {k: v.clone().requires_grad_(True) for k, v in T.to_torch(s).items()}
    g = g.clone().requires_grad_(True)
    pi = pi.clone().requires_grad_(True)
    m = torch.as_tensor(s["m"])
    mat = torch.as_tensor(s["mat"]).long()
    out = T.step_rk2_torch(st, m, mat, et, g, pi, pairs_at, H, dt, mirror_at=mirror_at,
                           wall=w.wall, t=t, box=box, periodic=per, pair_h=ph)
    s1_base, _, _, _ = O.step(cfg, s, t, dt_in=dt, d=d)
    for k in F8:
        assert np.abs(out[k].detach().numpy() - s1_base[k]).max() <= 1e-13 * (1 + np.abs(s1_base[k]).max()), k
    rng = np.random.default_rng(100)
    lam = {k: rng.standard_normal(w.n) for k in F8}
    J = sum((out[k] * torch.as_tensor(lam[k])).sum() for k in F8)
    grads = torch.autograd.grad(J, [st[k] for k in F8] + [g, pi])
    for trial in range(3):
        dd = {k: rng.standard_normal(w.n) for k in F8}
        dg = rng.standard_normal(len(w.eos))
        dpi = rng.standard_normal(len(w.eos)) * np.array([0.0 if e[0] == 0 else 1.0 for e in w.eos])
        pred = sum(float((grads[a].numpy() * dd[k]).sum()) for a, k in enumerate(F8))
        pred += float((grads[8].numpy() * dg).sum()) + float((grads[9].numpy() * dpi).sum())
        eps = 1e-6

        def J_at(sign):
            s2 = {k: (s[k] + sign * eps * dd[k]) if k in dd else s[k] for k in s}
            kw = dict(h=w.h, kappa=w.kappa, cfl=0.0, wall=w.wall, periodic=per, box=box,
                      integrator=1)
            kw.update(hm)
            c2 = O.make_cfg(_eos_shifted(w.eos, sign, eps, dg, dpi), **kw)
            s1, _, _, _ = O.step(c2, s2, t, dt_in=dt, d=d)
            return sum(float((s1[k] * lam[k]).sum()) for k in F8)

        fd = (J_at(1) - J_at(-1)) / (2 * eps)
        assert abs(fd - pred) <= 1e-6 * max(abs(pred), 1.0), (trial, fd, pred)


def test_torch_rates_pair_h_periodic_piston_match_c_oracle():
    """Pair-h mode on periodic sides with the piston (each pair's own support, image and
    mirror partners through the images): the reference's rates against the C oracle's."""
    w = periodic_system(6, seed=13, wall=(0.2, 0.4))
    d = np.random.default_rng(14).uniform(0.8, 1.3, w.n)
    cfg = O.cfg_for(w, h_mode=1, kappa=1.936)
    s = O.state_from(w, cfg)
    s["d"] = d
    t = 0.3
    ref = O.rates(cfg, s, t=t, d=d)
    et, g, pi = tparams(w)
    ph = (1.936, d)
    pairs = T.pairs_of(cfg, s)
    assert float(pairs[2].abs().max()) > 0.0  # image partners present
    xw = 0.2 + 0.4 * t
    mir = T.mirror_pairs_of(s, 0.0, xw, box=w.box, periodic=6, pair_h=ph)
    assert float(mir[2].abs().max()) > 0.0  # mirror partners through the images
    out = T.rates_torch(T.to_torch(s), torch.as_tensor(s["m"]), torch.as_tensor(s["mat"]).long(),
                        et, g, pi, pairs, 0.0, mirror=mir, wall=(xw, 0.4), pair_h=ph)
    for k, v in zip(("drho", "dvx", "dvy", "dvz", "dE"), out):
        scale = np.abs(ref[k]).max()
        assert np.abs(v.numpy() - ref[k]).max() <= 1e-13 * scale, k
    # the step (reflections, the wrap across the periodic faces)
    dt = 0.2
    cfg0 = O.cfg_for(w, h_mode=1, kappa=1.936, cfl=0.0)
    s1, _, _, _ = O.step(cfg0, s, t, dt_in=dt, d=d)
    out = T.step_torch(T.to_torch(s), torch.as_tensor(s["m"]), torch.as_tensor(s["mat"]).long(),
                       et, g, pi, pairs, 0.0, dt, mirror=mir, wall=(0.2, 0.4), t=t, box=w.box,
                       periodic=6, pair_h=ph)
    for k in F8:
        assert np.abs(out[k].numpy() - s1[k]).max() <= 1e-13 * (1 + np.abs(s1[k]).max()), k
