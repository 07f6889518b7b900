"""Seeded synthetic node sets shaped like the paper's 2D/3D irregular-domain cases.

This module is shared input tooling: the CPU oracle, the GPU tests and the
benchmark all draw their inputs from it.  It holds geometry only (lattices,
jitter, boundary samplers, inside tests) and none of the method's arithmetic:
no stencil selection, no weights, no sparse assembly.

Recipe (the paper's own fills, GeneralFill / GrainDropFill of Sec. 3.1, are
only cited there, so a jittered lattice stands in for them):

* interior: lattice points k*h (integer k) plus an independent uniform jitter
  U(-h/4, h/4) per coordinate, drawn for the whole bounding lattice in C order
  from ``numpy.random.default_rng(seed)``; a jittered point is kept when its
  distance to the domain boundary is at least h/2;
* boundary: deterministic samples at spacing about h (equispaced circles,
  the surface lattice of a cube, Fibonacci lattices on spheres, polygon edges,
  a ring-by-ring torus surface);
* node order: interior nodes first (lattice C order), then boundary nodes.

Every function returns a :class:`NodeSet`.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN_ANGLE = math.pi * (3.0 - math.sqrt(5.0))


@dataclass
class NodeSet:
    X: np.ndarray            # [N, d] float64, row-major
    is_boundary: np.ndarray  # [N] bool
    h: np.ndarray            # [N] float64 generator spacing of the node's domain
    d: int
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.X.shape[0])


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------

def _lattice(d: int, lo: np.ndarray, hi: np.ndarray, h: float) -> np.ndarray:
    """All points k*h (integer k) inside the box [lo, hi], C order."""
    axes = [np.arange(math.ceil(lo[a] / h - 1e-9), math.floor(hi[a] / h + 1e-9) + 1) * h
            for a in range(d)]
    grids = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.reshape(-1) for g in grids], axis=1)


def _jittered_interior(d, lo, hi, h, dist_fn, rng, chunk=1 << 22):
    """Jittered lattice points whose boundary distance is >= h/2."""
    P = _lattice(d, np.asarray(lo, float), np.asarray(hi, float), h)
    P = P + rng.uniform(-0.25 * h, 0.25 * h, size=P.shape)
    keep = np.empty(P.shape[0], dtype=bool)
    for s in range(0, P.shape[0], chunk):
        keep[s:s + chunk] = dist_fn(P[s:s + chunk]) >= 0.5 * h
    return P[keep]


def circle_points(center, radius, h):
    M = max(3, int(round(2.0 * math.pi * radius / h)))
    t = 2.0 * math.pi * np.arange(M) / M
    return np.stack([center[0] + radius * np.cos(t), center[1] + radius * np.sin(t)], axis=1)


def fibonacci_sphere(center, radius, h):
    M = max(4, int(round(4.0 * math.pi * radius * radius / (h * h))))
    k = np.arange(M)
    z = 1.0 - (2.0 * k + 1.0) / M
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    th = k * GOLDEN_ANGLE
    return np.stack([center[0] + radius * rho * np.cos(th),
                     center[1] + radius * rho * np.sin(th),
                     center[2] + radius * z], axis=1)


def cube_surface_lattice(h, lo=0.0, hi=1.0):
    """Lattice points of [lo,hi]^3 with at least one coordinate on a face (each once)."""
    k = int(round((hi - lo) / h))
    ax = lo + np.arange(k + 1) * h
    g = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1).reshape(-1, 3)
    idx = np.stack(np.meshgrid(*(np.arange(k + 1),) * 3, indexing="ij"), axis=-1).reshape(-1, 3)
    on = np.any((idx == 0) | (idx == k), axis=1)
    return g[on]


def polygon_edges(verts, h):
    """Points at spacing about h along a closed polygon (each vertex once)."""
    out = []
    nv = len(verts)
    for a in range(nv):
        p, q = np.asarray(verts[a], float), np.asarray(verts[(a + 1) % nv], float)
        L = float(np.linalg.norm(q - p))
        M = max(1, int(round(L / h)))
        t = np.arange(M) / M
        out.append(p[None, :] + t[:, None] * (q - p)[None, :])
    return np.concatenate(out, axis=0)


def _seg_dist(P, a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    ab = b - a
    t = np.clip(((P - a) @ ab) / (ab @ ab), 0.0, 1.0)
    return np.linalg.norm(P - (a + t[:, None] * ab), axis=1)


def torus_surface(center, R, r, h):
    """Ring-by-ring samples of the torus surface; ring density follows the area element."""
    Nv = max(3, int(round(2.0 * math.pi * r / h)))
    out = []
    for j in range(Nv):
        v = 2.0 * math.pi * j / Nv
        rho = R + r * math.cos(v)
        Nu = max(3, int(round(2.0 * math.pi * rho / h)))
        u = 2.0 * math.pi * np.arange(Nu) / Nu
        out.append(np.stack([center[0] + rho * np.cos(u),
                             center[1] + rho * np.sin(u),
                             np.full(Nu, center[2] + r * math.sin(v))], axis=1))
    return np.concatenate(out, axis=0)


def _make(interior, boundary, h, d, **meta):
    X = np.ascontiguousarray(np.concatenate([interior, boundary], axis=0), dtype=np.float64)
    isb = np.zeros(X.shape[0], dtype=bool)
    isb[interior.shape[0]:] = True
    return NodeSet(X=X, is_boundary=isb, h=np.full(X.shape[0], float(h)), d=d, meta=dict(meta))


# --------------------------------------------------------------------------
# domains
# --------------------------------------------------------------------------

def disk(h: float, seed: int, center=(0.0, 0.0), radius=1.0) -> NodeSet:
    """Unit disk: jittered lattice + equispaced circle nodes."""
    rng = np.random.default_rng(seed)
    c = np.asarray(center, float)
    dist = lambda P: radius - np.linalg.norm(P - c, axis=1)
    inner = _jittered_interior(2, c - radius, c + radius, h, dist, rng)
    return _make(inner, circle_points(c, radius, h), h, 2, domain="disk", seed=seed)


def annulus(h: float, seed: int, d: int = 2, r_in=0.5, r_out=1.0) -> NodeSet:
    """B(0, r_out) minus B(0, r_in) in 2D or 3D (the paper's Poisson benchmark domain)."""
    rng = np.random.default_rng(seed)
    dist = lambda P: np.minimum(r_out - np.linalg.norm(P, axis=1), np.linalg.norm(P, axis=1) - r_in)
    inner = _jittered_interior(d, -r_out * np.ones(d), r_out * np.ones(d), h, dist, rng)
    z = np.zeros(d)
    if d == 2:
        bnd = np.concatenate([circle_points(z, r_out, h), circle_points(z, r_in, h)])
    else:
        bnd = np.concatenate([fibonacci_sphere(z, r_out, h), fibonacci_sphere(z, r_in, h)])
    return _make(inner, bnd, h, d, domain="annulus", seed=seed)


def cube_minus_balls(h: float, seed: int, centers, radii) -> NodeSet:
    """[0,1]^3 minus a union of balls: jittered lattice, face lattice, Fibonacci spheres."""
    rng = np.random.default_rng(seed)
    C = np.asarray(centers, float).reshape(-1, 3)
    Rr = np.asarray(radii, float).reshape(-1)

    def dist(P):
        dd = np.minimum(P, 1.0 - P).min(axis=1)
        for c, r in zip(C, Rr):
            dd = np.minimum(dd, np.linalg.norm(P - c, axis=1) - r)
        return dd

    inner = _jittered_interior(3, np.zeros(3), np.ones(3), h, dist, rng)
    faces = cube_surface_lattice(h)
    # face nodes inside any ball are not on the domain boundary
    keep = np.ones(faces.shape[0], dtype=bool)
    for c, r in zip(C, Rr):
        keep &= np.linalg.norm(faces - c, axis=1) > r
    parts = [faces[keep]]
    for b, (c, r) in enumerate(zip(C, Rr)):
        S = fibonacci_sphere(c, r, h)
        ok = np.all((S > 0.0) & (S < 1.0), axis=1)
        for b2, (c2, r2) in enumerate(zip(C, Rr)):
            if b2 != b:
                ok &= np.linalg.norm(S - c2, axis=1) > r2
        parts.append(S[ok])
    return _make(inner, np.concatenate(parts), h, 3, domain="cube_minus_balls", seed=seed)


def cube_minus_sphere(h: float, seed: int) -> NodeSet:
    """[0,1]^3 minus the ball of radius 0.3 at the centre."""
    ns = cube_minus_balls(h, seed, [(0.5, 0.5, 0.5)], [0.3])
    ns.meta["domain"] = "cube_minus_sphere"
    return ns


def random_balls(seed: int, count=64, rmin=0.02, rmax=0.08, lo=0.1, hi=0.9):
    """Centres U[lo,hi]^3 and radii U[rmin,rmax] (overlaps allowed); drawn before the fill."""
    rng = np.random.default_rng(seed)
    centers = rng.uniform(lo, hi, size=(count, 3))
    radii = rng.uniform(rmin, rmax, size=count)
    return centers, radii


def disk_with_holes(h: float, seed: int, n_holes=3, r_hole=0.2, cmax=0.6, gap=0.1) -> NodeSet:
    """Unit disk minus holes of radius r_hole; centres |c| <= cmax, pairwise gap >= gap."""
    rng = np.random.default_rng(seed)
    cs = []
    while len(cs) < n_holes:
        c = rng.uniform(-cmax, cmax, size=2)
        if np.linalg.norm(c) > cmax:
            continue
        if all(np.linalg.norm(c - o) >= 2 * r_hole + gap for o in cs):
            cs.append(c)
    cs = np.asarray(cs)

    def dist(P):
        dd = 1.0 - np.linalg.norm(P, axis=1)
        for c in cs:
            dd = np.minimum(dd, np.linalg.norm(P - c, axis=1) - r_hole)
        return dd

    inner = _jittered_interior(2, -np.ones(2), np.ones(2), h, dist, rng)
    bnd = [circle_points(np.zeros(2), 1.0, h)] + [circle_points(c, r_hole, h) for c in cs]
    return _make(inner, np.concatenate(bnd), h, 2, domain="disk_with_holes", seed=seed,
                 hole_centers=cs.tolist())


L_SHAPE = [(0.0, 0.0), (1.0, 0.0), (1.0, 0.5), (0.5, 0.5), (0.5, 1.0), (0.0, 1.0)]


def l_shape(h: float, seed: int) -> NodeSet:
    """[0,1]^2 minus [1/2,1]^2."""
    rng = np.random.default_rng(seed)
    V = L_SHAPE

    def dist(P):
        inside = np.all((P >= 0.0) & (P <= 1.0), axis=1) & ~((P[:, 0] > 0.5) & (P[:, 1] > 0.5))
        dd = np.full(P.shape[0], np.inf)
        for a in range(len(V)):
            dd = np.minimum(dd, _seg_dist(P, V[a], V[(a + 1) % len(V)]))
        return np.where(inside, dd, -dd)

    inner = _jittered_interior(2, np.zeros(2), np.ones(2), h, dist, rng)
    return _make(inner, polygon_edges(V, h), h, 2, domain="l_shape", seed=seed)


def torus(h: float, seed: int, center=(0.5, 0.5, 0.5), R=0.35, r=0.15) -> NodeSet:
    """Solid torus (axis z)."""
    rng = np.random.default_rng(seed)
    c = np.asarray(center, float)

    def dist(P):
        q = P - c
        rho = np.sqrt(q[:, 0] ** 2 + q[:, 1] ** 2)
        return r - np.sqrt((rho - R) ** 2 + q[:, 2] ** 2)

    ext = np.array([R + r, R + r, r])
    inner = _jittered_interior(3, c - ext, c + ext, h, dist, rng)
    return _make(inner, torus_surface(c, R, r, h), h, 3, domain="torus", seed=seed)


def unit_square_grid(h: float) -> NodeSet:
    """Regular grid G_h over [0,1]^2 (the Laplacian-error study of Sec. 3.2)."""
    k = int(round(1.0 / h))
    ax = np.arange(k + 1) * (1.0 / k)
    g = np.stack(np.meshgrid(ax, ax, indexing="ij"), axis=-1).reshape(-1, 2)
    idx = np.stack(np.meshgrid(np.arange(k + 1), np.arange(k + 1), indexing="ij"), -1).reshape(-1, 2)
    isb = np.any((idx == 0) | (idx == k), axis=1)
    return NodeSet(X=np.ascontiguousarray(g), is_boundary=isb, h=np.full(g.shape[0], 1.0 / k), d=2,
                   meta=dict(domain="unit_square_grid"))


# --------------------------------------------------------------------------
# per-node stencil parameters (mixed batch)
# --------------------------------------------------------------------------

def n_monomials(d: int, P: int) -> int:
    """Dimension of the d-variate polynomials of total degree <= P: C(P+d, d)."""
    return math.comb(P + d, d)


def mixed_stencil_params(N: int, d: int, seed: int, Pmin=2, Pmax=4, n_hi=70, n_floor=12):
    """Per-node degree P ~ U{Pmin..Pmax}, then size n ~ U[max(n_floor, ceil(1.5 m)), n_hi].

    Drawn from default_rng(seed) in this order: all P, then all n.
    """
    rng = np.random.default_rng(seed)
    P = rng.integers(Pmin, Pmax + 1, size=N)
    m = np.array([n_monomials(d, p) for p in range(Pmax + 1)])[P]
    lo = np.maximum(n_floor, np.ceil(1.5 * m).astype(np.int64))
    n = lo + np.floor(rng.uniform(0.0, 1.0, size=N) * (n_hi - lo + 1)).astype(np.int64)
    return P.astype(np.int8), np.minimum(n, n_hi).astype(np.int64)


def offsets_from_sizes(n: np.ndarray) -> np.ndarray:
    """Exclusive prefix sum of stencil sizes, int64, length N+1."""
    off = np.zeros(n.shape[0] + 1, dtype=np.int64)
    np.cumsum(n, out=off[1:])
    return off


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

DISK_H = 0.0404          # about 2,000 nodes in the unit disk
CUBE_SPHERE_H = 1.0 / 106  # about 1.1M nodes in [0,1]^3 minus B(c, 0.3)
LARGE3D_H = 1.0 / 256    # about 16M nodes in [0,1]^3 minus 64 balls


def workload(name: str, h: float | None = None, seed: int | None = None) -> dict:
    """Named synthetic workloads.

    disk2d        : unit disk, n=15, degree 2, ops lap,dx,dy (seed 1001)
    cube_sphere3d : [0,1]^3 minus B(c,0.3), n=35, degree 3, ops lap,dx,dy,dz (seed 1002)
    mixed         : four 2D/3D domains, per-node n and degree (seed 1003)
    learned2d     : disk training sets, n=15, degree 2, lap only (seeds 4,000,000+k)
    large3d       : [0,1]^3 minus 64 random balls, n=65, degree 4, lap + gradient (seed 1005)

    ``h`` overrides the spacing (coarser copies of a workload for parity tests).
    """
    if name == "disk2d":
        ns = disk(h or DISK_H, 1001 if seed is None else seed)
        return dict(nodes=[ns], n=15, P=2, ops=("lap", "dx", "dy"))
    if name == "cube_sphere3d":
        ns = cube_minus_sphere(h or CUBE_SPHERE_H, 1002 if seed is None else seed)
        return dict(nodes=[ns], n=35, P=3, ops=("lap", "dx", "dy", "dz"))
    if name == "large3d":
        s = 1005 if seed is None else seed
        C, R = random_balls(s)
        ns = cube_minus_balls(h or LARGE3D_H, s + 1, C, R)
        return dict(nodes=[ns], n=65, P=4, ops=("lap", "dx", "dy", "dz"))
    if name == "learned2d":
        ns = disk(h or DISK_H, 4_000_000 if seed is None else seed)
        return dict(nodes=[ns], n=15, P=2, ops=("lap",))
    raise KeyError(name)


def mixed_domains(target_per_domain: int, seed: int = 1003):
    """The four mixed-batch domains, each scaled to about target_per_domain nodes.

    Returns a list of (NodeSet, P[N] int8, n[N] int64); per-node parameters use
    seed*10 + domain_id.
    """
    out = []
    # 2D: disk minus 3 holes (area 0.88*pi), L-shape (area 0.75)
    h0 = math.sqrt(0.88 * math.pi / target_per_domain)
    h1 = math.sqrt(0.75 / target_per_domain)
    # 3D: cube minus B(c,0.3) (volume 1 - 4/3 pi 0.027), torus (2 pi^2 R r^2)
    h2 = ((1.0 - 4.0 / 3.0 * math.pi * 0.027) / target_per_domain) ** (1.0 / 3.0)
    h3 = ((2.0 * math.pi ** 2 * 0.35 * 0.15 ** 2) / target_per_domain) ** (1.0 / 3.0)
    doms = [disk_with_holes(h0, seed * 10 + 0), l_shape(h1, seed * 10 + 1),
            cube_minus_sphere(h2, seed * 10 + 2), torus(h3, seed * 10 + 3)]
    for k, ns in enumerate(doms):
        P, n = mixed_stencil_params(ns.N, ns.d, seed * 10 + 4 + k)
        n = np.minimum(n, ns.N)
        out.append((ns, P, n))
    return out


def surrogate_init(seed: int, layers=((30, 128), (128, 128), (128, 128), (128, 15))) -> dict:
    """Seeded Xavier-uniform initial weights (bound sqrt(6/(fan_in+fan_out))), zero biases.

    Random draws only; W1..W4 drawn in that order from default_rng(seed), each [out, in].
    """
    rng = np.random.default_rng(seed)
    p = {}
    for L, (fi, fo) in enumerate(layers, start=1):
        a = math.sqrt(6.0 / (fi + fo))
        p[f"W{L}"] = rng.uniform(-a, a, size=(fo, fi))
        p[f"b{L}"] = np.zeros(fo)
    return p
