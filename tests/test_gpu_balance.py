"""GPU parity of the Voronoi balancer (csph_balance_stats, csph_balance_move)
against the numpy oracle (oracle/balance.py): loads and touching-subdomain
bits bit-exact, centres within the fixed-point resolution, generator moves
within 1e-12 relative, and a short static balancing run step by step."""
import numpy as np
import pytest
import torch

import csph_inputs as ci
from oracle import balance as B
import paper_1805_05128_amd as P

pytestmark = pytest.mark.gpu
DEV = "cuda"


def t64(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float64), device=DEV)


def t32(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.int32), device=DEV)


def cloud(n, K, seed, box=40.0, flat=False):
    w = ci.random_cloud(n, seed=seed, box=box)
    if flat:
        w.z = np.full(n, 0.5)
    sites = ci.voronoi_sites(K, seed, (box, box, 0.0 if flat else box))
    if flat:
        sites[:, 2] = 0.5
    return w, sites


def check_stats(w, sites, dsh, nbr=None, owner=None):
    K = sites.shape[0]
    if owner is None:
        owner = B.assign(w.x, w.y, w.z, sites)
    ref = B.stats(w.x, w.y, w.z, owner, sites, dsh, nbr)
    got = P.csph_balance_stats(t64(w.x), t64(w.y), t64(w.z), t32(owner), t64(sites), dsh,
                               nbr_count=None if nbr is None else t32(nbr))
    torch.cuda.synchronize()
    assert np.array_equal(got["particles"].cpu().numpy(), ref["particles"])
    if nbr is not None:
        assert np.array_equal(got["pairs"].cpu().numpy(), ref["pairs"])
    c = got["centre"].cpu().numpy()
    assert np.all(np.abs(c - ref["centre"]) <= 1e-9 + 1e-13 * np.abs(ref["centre"])), \
        np.abs(c - ref["centre"]).max()
    adj = P.adjacency_matrix(got["adjacency"], K).numpy()
    assert np.array_equal(adj, ref["adjacency"])
    return got, ref


@pytest.mark.parametrize("K", [1, 3, 64, 512])
def test_stats_random_cloud(K):
    n = 30000
    print(f"[case] stats cloud n={n} K={K}", flush=True)
    w, sites = cloud(n, K, seed=5)
    nbr = np.random.default_rng(K).integers(0, 200, n)
    check_stats(w, sites, dsh=2.0, nbr=nbr)


def test_stats_lattice_split_and_ignored_owners():
    w = ci.jittered_block(20, 20, 20, seed=1, amp=0.0)
    sites = np.array([[5.0, 10.0, 10.0], [15.0, 10.0, 10.0], [10.0, 30.0, 10.0]])
    print("[case] stats lattice split", flush=True)
    got, ref = check_stats(w, sites, dsh=1.0)
    assert got["particles"].cpu().tolist() == [4000, 4000, 0]
    # the empty subdomain keeps its generator as centre
    assert got["centre"].cpu().numpy()[2].tolist() == [10.0, 30.0, 10.0]
    owner = B.assign(w.x, w.y, w.z, sites)
    owner[::7] = -1
    owner[1::11] = 3
    check_stats(w, sites, dsh=1.0, owner=owner)


def test_stats_no_particles():
    sites = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    e = np.zeros(0)
    got = P.csph_balance_stats(t64(e), t64(e), t64(e), t32(np.zeros(0)), t64(sites), 1.0)
    assert got["particles"].cpu().tolist() == [0, 0]
    assert np.array_equal(got["centre"].cpu().numpy(), sites)
    assert not P.adjacency_matrix(got["adjacency"], 2).any()


def test_stats_large_cloud():
    n, K = 400000, 64
    print(f"[case] stats cloud n={n} K={K}", flush=True)
    w, sites = cloud(n, K, seed=9, box=80.0)
    check_stats(w, sites, dsh=3.0, nbr=np.random.default_rng(0).integers(50, 130, n))


@pytest.mark.parametrize("flat,sigma,theta", [(True, 0.5, 0.25), (False, 0.5, 0.25),
                                              (True, 1.0, 0.0), (False, 0.0, 1.0)])
def test_move_matches_oracle(flat, sigma, theta):
    n, K = 20000, 24
    print(f"[case] move flat={flat} sigma={sigma} theta={theta}", flush=True)
    w, sites = cloud(n, K, seed=7, flat=flat)
    owner = B.assign(w.x, w.y, w.z, sites)
    st = B.stats(w.x, w.y, w.z, owner, sites, 3.0)
    loads = st["particles"]
    p = B.BalanceParams(sigma=sigma, theta=theta, gamma=1.0, dsh=3.0, load="particles")
    ref, ref_ms = B.move(sites, loads, st["centre"], st["adjacency"], p)
    gst = P.csph_balance_stats(t64(w.x), t64(w.y), t64(w.z), t32(owner), t64(sites), 3.0)
    new, ms = P.csph_balance_move(t64(sites), gst, P.BalanceParams(sigma=sigma, theta=theta,
                                                                   gamma=1.0, dsh=3.0,
                                                                   load="particles"))
    new = new.cpu().numpy()
    scale = np.abs(sites).max()
    assert np.abs(new - ref).max() <= 1e-12 * scale, np.abs(new - ref).max()
    assert abs(float(ms.item()) - ref_ms) <= 1e-11 * max(ref_ms, 1.0)


def test_static_disk_balancing_run():
    """Three generators bunched on one side of a jittered disk layer; ten assign/stats/move
    iterations on the GPU follow the oracle's iterations."""
    R = 30.0
    g = np.arange(-R, R + 1.0)
    X, Y = np.meshgrid(g, g, indexing="ij")
    m = X ** 2 + Y ** 2 <= R * R
    rng = np.random.default_rng(4)
    x = X[m] + rng.uniform(-0.01, 0.01, m.sum())
    y = Y[m] + rng.uniform(-0.01, 0.01, m.sum())
    z = np.full(x.size, 0.5)
    sites = np.array([[18.0, 2.0, 0.5], [20.0, -3.0, 0.5], [22.0, 4.0, 0.5]])
    p = B.BalanceParams(sigma=0.5, theta=0.25, gamma=1.0, dsh=3.0, load="particles")
    hist = B.iterate(x, y, z, sites, p, 10)
    gp = P.BalanceParams(sigma=0.5, theta=0.25, gamma=1.0, dsh=3.0, load="particles")
    xs, ys, zs = t64(x), t64(y), t64(z)
    gs = t64(sites)
    print("[case] disk run 10 iterations", flush=True)
    for it, (s_ref, l_ref, ms_ref) in enumerate(hist):
        assert np.abs(gs.cpu().numpy() - s_ref).max() <= 1e-9, it
        owner, part, _ = P.voronoi_assign(xs, ys, zs, gs)
        st = P.csph_balance_stats(xs, ys, zs, owner, gs, gp.dsh)
        assert np.array_equal(st["particles"].cpu().numpy(), l_ref), it
        gs, ms = P.csph_balance_move(gs, st, gp)
        assert abs(float(ms.item()) - ms_ref) <= 1e-9 * max(ms_ref, 1.0), it
