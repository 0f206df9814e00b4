"""Pins of the balancer oracle (oracle/balance.py) against closed forms, the
cases the paper spells out for fig. 4 (two-body magnitudes; no net rotation
of the heavy generator, rotation of the light ones by pi/3 * dL / sum L),
geometric identities, and a brute-force static balancing run."""
import math

import numpy as np
import pytest

from oracle import balance as B


def ring(angles_deg, R=1.0, centre=(0.0, 0.0, 0.0)):
    a = np.radians(np.asarray(angles_deg, np.float64))
    c = np.asarray(centre, np.float64)
    return np.stack([c[0] + R * np.cos(a), c[1] + R * np.sin(a), np.full(a.shape, c[2])], 1)


def full_adj(K):
    return ~np.eye(K, dtype=bool)


def angle_deg(v):
    return math.degrees(math.atan2(v[1], v[0])) % 360.0


# ------------------------------------------------------------------ geometry

def test_rotation_matrix_is_a_right_handed_rotation():
    M = B.rotation_matrix([0, 0, 2.0], math.pi / 2)
    assert np.allclose(M @ [1.0, 0, 0], [0, 1.0, 0], atol=1e-15)
    rng = np.random.default_rng(0)
    for _ in range(5):
        M = B.rotation_matrix(rng.standard_normal(3), rng.uniform(-3, 3))
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(M) - 1.0) < 1e-14


def test_circumcentre_right_triangle_and_random():
    o = B.circumcentre([0, 0, 0], [4.0, 0, 0], [0, 3.0, 0])
    assert np.allclose(o, [2.0, 1.5, 0.0], atol=1e-15)  # midpoint of the hypotenuse
    rng = np.random.default_rng(1)
    for _ in range(10):
        a, b, c = rng.standard_normal((3, 3))
        o = B.circumcentre(a, b, c)
        r = [np.linalg.norm(o - p) for p in (a, b, c)]
        assert max(r) - min(r) < 1e-12 * max(r)
        assert abs(np.dot(np.cross(b - a, c - a), o - a)) < 1e-12 * max(r) ** 3
    assert B.circumcentre([0, 0, 0], [1.0, 0, 0], [2.0, 0, 0]) is None


# ------------------------------------------------------------------ eq. BalancingOffset

def test_equal_loads_give_no_displacement():
    rng = np.random.default_rng(2)
    sites = rng.uniform(0, 10, (6, 3))
    p = B.BalanceParams(sigma=0.5, theta=0.0, gamma=1.0, dsh=3.0)
    dg = B.displacement(sites, np.full(6, 7.0), full_adj(6), p)
    assert np.array_equal(dg, np.zeros_like(dg))
    new, ms = B.move(sites, np.full(6, 7.0), sites * 0.0, full_adj(6), p)
    assert np.array_equal(new, sites) and ms == 0.0


def test_two_sites_heavy_recedes_light_follows():
    sites = np.array([[0.0, 0, 0], [4.0, 0, 0]])
    p = B.BalanceParams(sigma=0.0, theta=0.0, gamma=1.0, dsh=2.0)
    dg = B.displacement(sites, np.array([3.0, 1.0]), full_adj(2), p)
    # D (L0 - L1)/(L0 + L1) = 2 * 2/4 = 1 along g_01 = g_0 - g_1 = -x; site 1 by -1 along +x
    assert np.allclose(dg, [[-1.0, 0, 0], [-1.0, 0, 0]], atol=0, rtol=0)
    # the bisector moves from x = 2 to x = 1: the heavy subdomain shrinks
    new = sites + dg
    assert 0.5 * (new[0, 0] + new[1, 0]) == 1.0


def test_fig4b_two_body_magnitudes():
    """Heavy site 0 between light sites 1, 2 (L1 = L2): |dg_1| = |dg_2| = D dL/(Lh+Ll) from
    the pair with 0 only; dg_0 = D dL/(Lh+Ll) (u_01 + u_02)."""
    sites = ring([90.0, 210.0, 330.0], R=5.0)
    Lh, Ll, D = 0.5, 0.25, 1.5
    dg = B.two_body(sites, np.array([Lh, Ll, Ll]), full_adj(3), D)
    f = D * (Lh - Ll) / (Lh + Ll)
    u = lambda a, b: (sites[a] - sites[b]) / np.linalg.norm(sites[a] - sites[b])
    assert np.allclose(dg[0], f * (u(0, 1) + u(0, 2)), atol=1e-15)
    assert np.allclose(dg[1], -f * u(1, 0), atol=1e-15)
    assert abs(np.linalg.norm(dg[2]) - f) < 1e-15


# ------------------------------------------------------------------ eq. BalancingOffsetRot

def test_fig4c_three_body_rotation():
    """sigma = 1: the heavy generator does not turn (alpha_0 ~ 0 for equal light loads); each
    light generator turns about the circumcentre by pi/3 (Lh - Ll)/sum L towards the heavy
    one, keeping its distance to the circumcentre."""
    c = (3.0, -2.0, 1.0)
    sites = ring([90.0, 210.0, 330.0], R=2.0, centre=c)
    Lh, Ll = 0.5, 0.25
    p = B.BalanceParams(sigma=1.0, theta=0.0, gamma=1.0, dsh=100.0)
    new, _ = B.move(sites, np.array([Lh, Ll, Ll]), sites, full_adj(3), p)
    assert np.allclose(new[0], sites[0], atol=1e-14)
    alpha = math.degrees(math.pi / 3 * (Lh - Ll) / (Lh + 2 * Ll))
    for k, a0 in ((1, 210.0), (2, 330.0)):
        v = new[k] - np.asarray(c)
        assert abs(np.linalg.norm(v) - 2.0) < 1e-14
        assert abs(v[2]) < 1e-14
        want = a0 - alpha if k == 1 else a0 + alpha   # towards site 0 at 90 degrees
        assert abs(angle_deg(v) - want) < 1e-11


def test_three_body_sector_model_contraction():
    """Generators on a circle about the common point, loads = sector angles: the rule turns
    generator k by (pi/3)(L_l - L_m)/sum L, so each inter-generator gap error shrinks by 3/4
    per iteration (closed form of the sector model; the fixed point is 120 degrees)."""
    ang = np.array([90.0, 170.0, 330.0])
    p = B.BalanceParams(sigma=1.0, theta=0.0, gamma=1.0, dsh=100.0)
    for it in range(3):
        gaps = np.diff(np.r_[ang, ang[0] + 360.0])        # a (0->1), b (1->2), c (2->0)
        sectors = 0.5 * (gaps + np.roll(gaps, 1))         # s_k = (gap before + gap after)/2
        new, _ = B.move(ring(ang), sectors, ring(ang), full_adj(3), p)
        ang2 = np.array([angle_deg(v) for v in new])
        gaps2 = np.diff(np.r_[ang2, ang2[0] + 360.0])
        assert np.allclose(gaps2 - 120.0, 0.75 * (gaps - 120.0), atol=1e-9), (it, gaps, gaps2)
        ang = ang2


def test_three_body_shift_is_capped():
    sites = ring([90.0, 100.0, 330.0], R=50.0)
    p = B.BalanceParams(sigma=1.0, theta=0.0, gamma=1.0, dsh=0.5)
    dg = B.displacement(sites, np.array([100.0, 1.0, 1.0]), full_adj(3), p)
    nrm = np.linalg.norm(dg, axis=1)
    assert nrm[0] < 1e-13                     # equal light loads: the heavy one does not turn
    assert np.allclose(nrm[1:], 0.5, atol=1e-14)


# ------------------------------------------------------------------ eq. TotalOffset

def test_cumulative_movement_limits():
    rng = np.random.default_rng(3)
    sites = rng.uniform(0, 10, (4, 3))
    centre = rng.uniform(0, 10, (4, 3))
    loads = rng.uniform(1, 5, 4)
    follow, ms = B.move(sites, loads, centre, full_adj(4), B.BalanceParams(theta=1.0))
    assert np.array_equal(follow, centre)
    assert abs(ms - np.linalg.norm(centre - sites, axis=1).sum()) < 1e-12
    static, ms0 = B.move(sites, loads, centre, full_adj(4), B.BalanceParams(theta=0.0, gamma=0.0))
    assert np.array_equal(static, sites) and ms0 == 0.0


# ------------------------------------------------------------------ statistics

def lattice_points(nx, ny, nz):
    g = np.stack(np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5, np.arange(nz) + 0.5,
                             indexing="ij"), -1).reshape(-1, 3)
    return g[:, 0].copy(), g[:, 1].copy(), g[:, 2].copy()


def test_stats_split_lattice():
    x, y, z = lattice_points(10, 10, 10)
    sites = np.array([[2.5, 5.0, 5.0], [7.5, 5.0, 5.0]])
    own = B.assign(x, y, z, sites)
    st = B.stats(x, y, z, own, sites, dsh=1.0, nbr_count=np.full(x.size, 3))
    assert st["particles"].tolist() == [500, 500]
    assert st["pairs"].tolist() == [1500, 1500]
    assert np.array_equal(st["centre"], [[2.5, 5.0, 5.0], [7.5, 5.0, 5.0]])
    assert st["adjacency"].tolist() == [[False, True], [True, False]]
    # the nearest particles are 0.5 from the bisector x = 5
    st = B.stats(x, y, z, own, sites, dsh=0.4)
    assert not st["adjacency"].any()


def test_stats_three_in_a_row_touch_only_neighbours():
    x, y, z = lattice_points(12, 4, 4)
    sites = np.array([[1.5, 2.0, 2.0], [6.0, 2.0, 2.0], [10.5, 2.0, 2.0]])
    own = B.assign(x, y, z, sites)
    adj = B.stats(x, y, z, own, sites, dsh=1.0)["adjacency"]
    assert adj.tolist() == [[False, True, False], [True, False, True], [False, True, False]]


def test_assign_ties_to_smaller_index():
    own = B.assign(np.array([5.0]), np.array([0.0]), np.array([0.0]),
                   np.array([[4.0, 0, 0], [6.0, 0, 0]]))
    assert own.tolist() == [0]


# ------------------------------------------------------------------ static balancing run

@pytest.mark.parametrize("sigma,theta", [(0.0, 0.0), (1.0, 0.0), (0.5, 0.0), (0.5, 0.25)])
def test_disk_balances_from_a_bad_start(sigma, theta):
    """A disk of material at rest (one lattice layer, radius 30) split by three generators
    bunched on one side: every combination of terms equalises the particle loads to within
    1 %.  (The paper's iteration counts come from a start shown only in a figure and are not
    pinned.)"""
    R = 30.0
    g = np.arange(-R, R + 1.0)
    X, Y = np.meshgrid(g, g, indexing="ij")
    m = X ** 2 + Y ** 2 <= R * R
    x, y = X[m].astype(float), Y[m].astype(float)
    z = np.zeros_like(x)
    sites = np.array([[18.0, 2.0, 0.0], [20.0, -3.0, 0.0], [22.0, 4.0, 0.0]])
    p = B.BalanceParams(sigma=sigma, theta=theta, gamma=1.0, dsh=3.0, load="particles")
    hist = B.iterate(x, y, z, sites, p, 80)
    L0, L = hist[0][1], hist[-1][1]
    assert L0.max() / L0.min() > 5.0
    assert L.max() / L.min() < 1.01
