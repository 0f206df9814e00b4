"""Oracle of the Voronoi load balancer (test infrastructure only).

Plain numpy FP64, written from sec. 3 of the paper:

* subdomain statistics: particle and pair loads, geometric centres
  (eq. VoronoiGeomCenters), and which subdomains touch (share a boundary
  layer of half width D^sh inside the material);
* the two-body balancing displacement (eq. BalancingOffset);
* the three-body rotation term for triplets of touching subdomains
  (eqs. BalancingOffsetPlusRot and BalancingOffsetRot), rotations about the
  circumcentre of the three generators, shift length capped at D^sh;
* the cumulative generator movement (eq. TotalOffset) and the convergence
  measure sum_k |g_k' - g_k| (eq. VDConvergence).

Readings where the paper leaves a choice (each is listed with the design
notes of the repository):

* g_kl = g_k - g_l, so a heavier subdomain's generator moves away from a
  lighter neighbour and the lighter one moves towards it: the boundary
  moves into the heavy subdomain, the attraction the paper describes.
* The double sum over l and m of three-body terms takes every triplet of
  mutually touching subdomains once (l < m); the two rotations are applied
  as written, first about c_k x c_l by alpha_l, then about c_k x c_m by
  alpha_m.  Collinear triplets (no circumcircle) contribute nothing.
* r_c + dr_c (centre plus mean Lagrangian displacement since the last
  rebalance) is the mean current position of the particles assigned at the
  last rebalance, since particles are not reassigned in between; a
  subdomain without particles uses its generator.
* L_k + L_l = 0 (both empty) gives no two-body term; a triplet with zero
  total load gives no three-body term.
* Two subdomains touch when some particle owned by one has the other as its
  nearest other generator and lies within D^sh of their bisector plane
  (symmetrised), i.e. the material has a boundary layer between them.
  Triplets are mutually touching triples.

The claim that the angle rule gives the 120 degree decomposition after one
iteration is not pinned: it depends on a geometry given only in a figure.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class BalanceParams:
    sigma: float = 0.5    # weight of three-body terms (eq. BalancingOffsetPlusRot)
    theta: float = 0.25   # weight of the material motion (eq. TotalOffset)
    gamma: float = 1.0    # scale of the balancing displacement (eq. TotalOffset)
    dsh: float = 3.0      # D^sh: exchange-layer half width; length factor and cap
    load: str = "pairs"   # "pairs" (directed interactions) or "particles"


# ------------------------------------------------------------------ statistics

def d2_to_sites(x, y, z, sites):
    """Squared distances [n, K], contraction-free FP64 in the order ((dx^2 + dy^2) + dz^2)."""
    dx = x[:, None] - sites[None, :, 0]
    dy = y[:, None] - sites[None, :, 1]
    dz = z[:, None] - sites[None, :, 2]
    return ((dx * dx) + (dy * dy)) + (dz * dz)


def stats(x, y, z, owner, sites, dsh, nbr_count=None):
    """Per-subdomain statistics of the current assignment ``owner``.

    Returns dict(particles int64 [K], pairs int64 [K], centre float64 [K, 3],
    adjacency bool [K, K]).  Owners outside [0, K) are ignored.
    """
    x, y, z = (np.asarray(a, np.float64) for a in (x, y, z))
    owner = np.asarray(owner, np.int64)
    sites = np.asarray(sites, np.float64).reshape(-1, 3)
    K = sites.shape[0]
    ok = (owner >= 0) & (owner < K)          # other entries are ignored
    if not ok.all():
        x, y, z, owner = x[ok], y[ok], z[ok], owner[ok]
        nbr_count = None if nbr_count is None else np.asarray(nbr_count)[ok]
    n = x.shape[0]
    parts = np.bincount(owner, minlength=K).astype(np.int64)
    pairs = np.zeros(K, np.int64)
    if nbr_count is not None:
        np.add.at(pairs, owner, np.asarray(nbr_count, np.int64))
    # eq. VoronoiGeomCenters: exact mean of the owned positions
    centre = sites.copy()
    for k in range(K):
        sel = owner == k
        if sel.any():
            cnt = int(sel.sum())
            centre[k] = [math.fsum(a[sel]) / cnt for a in (x, y, z)]
    adj = np.zeros((K, K), bool)
    if K > 1 and n > 0:
        d2 = d2_to_sites(x, y, z, sites)
        d2o = d2[np.arange(n), owner]
        d2m = d2.copy()
        d2m[np.arange(n), owner] = np.inf
        other = np.argmin(d2m, axis=1)          # nearest other generator, ties -> smaller k
        d2l = d2m[np.arange(n), other]
        g = sites[other] - sites[owner]
        gg = ((g[:, 0] * g[:, 0]) + (g[:, 1] * g[:, 1])) + (g[:, 2] * g[:, 2])
        # distance to the bisector plane = |d2l - d2o| / (2 |g_l - g_o|) < dsh, squared
        q = d2l - d2o
        near = (q * q) < (4.0 * (dsh * dsh)) * gg
        adj[owner[near], other[near]] = True
        adj = adj | adj.T
    return dict(particles=parts, pairs=pairs, centre=centre, adjacency=adj)


# ------------------------------------------------------------------ displacement

def rotation_matrix(axis, angle):
    """M(a, alpha): rotation by alpha about the unit vector along a (right hand)."""
    u = np.asarray(axis, np.float64)
    u = u / np.linalg.norm(u)
    ux = np.array([[0.0, -u[2], u[1]], [u[2], 0.0, -u[0]], [-u[1], u[0], 0.0]])
    return math.cos(angle) * np.eye(3) + math.sin(angle) * ux + (1.0 - math.cos(angle)) * np.outer(u, u)


def circumcentre(a, b, c):
    """Centre of the circle through a, b, c (in their plane), or None if collinear."""
    a, b, c = (np.asarray(v, np.float64) for v in (a, b, c))
    nrm = np.cross(b - a, c - a)
    if np.dot(nrm, nrm) <= 1e-24 * np.dot(b - a, b - a) * np.dot(c - a, c - a):
        return None
    # equidistant from a, b, c and in their plane
    A = np.array([2.0 * (b - a), 2.0 * (c - a), nrm])
    rhs = np.array([np.dot(b, b) - np.dot(a, a), np.dot(c, c) - np.dot(a, a), np.dot(nrm, a)])
    return np.linalg.solve(A, rhs)


def two_body(sites, loads, adj, dsh):
    """eq. BalancingOffset: sum over touching l of D^sh (L_k-L_l)/(L_k+L_l) g_kl/|g_kl|."""
    K = sites.shape[0]
    out = np.zeros((K, 3))
    for k in range(K):
        for l in range(K):
            if l == k or not adj[k, l]:
                continue
            s = loads[k] + loads[l]
            gkl = sites[k] - sites[l]
            nd = np.linalg.norm(gkl)
            if s == 0 or nd == 0.0:
                continue
            out[k] += dsh * (loads[k] - loads[l]) / s * gkl / nd
    return out


def three_body_terms(sites, loads, adj, k):
    """eq. BalancingOffsetRot summed over triplets (k, l, m), l < m, mutually touching."""
    K = sites.shape[0]
    tot = np.zeros(3)
    for l in range(K):
        if l == k or not adj[k, l]:
            continue
        for m in range(l + 1, K):
            if m == k or not adj[k, m] or not adj[l, m]:
                continue
            o = circumcentre(sites[k], sites[l], sites[m])
            S = loads[k] + loads[l] + loads[m]
            if o is None or S == 0:
                continue
            ck, cl, cm = sites[k] - o, sites[l] - o, sites[m] - o
            al = math.pi / 3.0 * (loads[l] - loads[k]) / S
            am = math.pi / 3.0 * (loads[m] - loads[k]) / S
            axl, axm = np.cross(ck, cl), np.cross(ck, cm)
            if np.linalg.norm(axl) == 0.0 or np.linalg.norm(axm) == 0.0:
                continue
            tot += -ck + rotation_matrix(axm, am) @ (rotation_matrix(axl, al) @ ck)
    return tot


def displacement(sites, loads, adj, p: BalanceParams):
    """eq. BalancingOffsetPlusRot with the three-body shift capped at D^sh."""
    sites = np.asarray(sites, np.float64).reshape(-1, 3)
    loads = np.asarray(loads, np.float64)
    two = two_body(sites, loads, adj, p.dsh)
    out = np.empty_like(two)
    for k in range(sites.shape[0]):
        t = three_body_terms(sites, loads, adj, k)
        nt = np.linalg.norm(t)
        if nt > p.dsh:
            t = t * (p.dsh / nt)
        out[k] = (1.0 - p.sigma) * two[k] + p.sigma * t
    return out


def move(sites, loads, centre, adj, p: BalanceParams):
    """eq. TotalOffset; returns (new sites [K, 3], sum_k |g_k' - g_k| of eq. VDConvergence)."""
    sites = np.asarray(sites, np.float64).reshape(-1, 3)
    dg = displacement(sites, loads, adj, p)
    new = (1.0 - p.theta) * (sites + p.gamma * dg) + p.theta * np.asarray(centre, np.float64)
    return new, float(sum(np.linalg.norm(new - sites, axis=1)))


def assign(x, y, z, sites):
    """eq. VoronoiDefinition with ties to the smaller index."""
    return np.argmin(d2_to_sites(x, y, z, np.asarray(sites, np.float64).reshape(-1, 3)), axis=1)


def iterate(x, y, z, sites, p: BalanceParams, iters, nbr_count=None):
    """Static balancing loop (material at rest): assign, measure, move.
    Returns the list of (sites, loads, move_sum) per iteration."""
    out = []
    sites = np.asarray(sites, np.float64).reshape(-1, 3)
    for _ in range(iters):
        own = assign(x, y, z, sites)
        st = stats(x, y, z, own, sites, p.dsh, nbr_count)
        loads = st["pairs"] if (p.load == "pairs" and nbr_count is not None) else st["particles"]
        new, ms = move(sites, loads, st["centre"], st["adjacency"], p)
        out.append((sites, loads, ms))
        sites = new
    return out
