"""Inputs and closed forms of the explicit heat problems used by the tests.

The heat example of Sec. 3.3.1: du/dt = lap u + 5 on a 2D domain with an outer
boundary carrying u = x (Dirichlet) and an inner circle with zero flux
(Neumann).  On the annulus r_in < r < 1 both steady states below solve
lap u = -5 exactly:

* inner circle Neumann (du/dr = 0 at r_in):
      u = 5/4 (1 - r^2) + (5 a^2 / 2) ln r + (r + a^2 / r) cos(theta) / (1 + a^2)
* inner circle Dirichlet with u = x there too:
      u = 5/4 (1 - r^2) + B ln r + x,  B = 5 (a^2 - 1) / (4 ln a)
with a = r_in.  The 5-point lattice Laplacian case has the discrete eigenmode
sin(pi x) sin(pi y) with eigenvalue -(8 / h^2) sin^2(pi h / 2).
"""
from __future__ import annotations

import math

import numpy as np

import nodesets as ns

INTERIOR, DIRICHLET, NEUMANN = 0, 1, 2


def annulus_heat(h: float, seed: int = 7, r_in: float = 0.5, neumann_inner: bool = True):
    """Annulus node set with node kinds, outward normals (inner circle) and g."""
    nd = ns.annulus(h, seed, d=2, r_in=r_in, r_out=1.0)
    X = nd.X
    r = np.linalg.norm(X, axis=1)
    mid = 0.5 * (r_in + 1.0)
    inner = nd.is_boundary & (r < mid)
    outer = nd.is_boundary & (r >= mid)
    kind = np.zeros(nd.N, dtype=np.uint8)
    kind[outer] = DIRICHLET
    kind[inner] = NEUMANN if neumann_inner else DIRICHLET
    normals = np.zeros((nd.N, 2))
    normals[inner] = -X[inner] / r[inner, None]   # out of the domain, into the hole
    g = np.zeros(nd.N)
    g[outer] = X[outer, 0]
    if not neumann_inner:
        g[inner] = X[inner, 0]
    return nd, kind, normals, g


def annulus_steady(X, r_in: float = 0.5, neumann_inner: bool = True):
    X = np.asarray(X)
    r = np.linalg.norm(X, axis=1)
    a = r_in
    if neumann_inner:
        return 1.25 * (1 - r * r) + 2.5 * a * a * np.log(r) + (r + a * a / r) * (X[:, 0] / r) / (1 + a * a)
    B = 5.0 * (a * a - 1.0) / (4.0 * math.log(a))
    return 1.25 * (1 - r * r) + B * np.log(r) + X[:, 0]


def lattice_5point(m: int):
    """m x m lattice on [0,1]^2 (h = 1/(m-1)), row-major.  Interior nodes carry the
    5-point stencil (self, +x, -x, +y, -y) with weights (-4, 1, 1, 1, 1)/h^2;
    boundary nodes a one-node stencil with weight 0 and kind DIRICHLET."""
    h = 1.0 / (m - 1)
    xs = np.arange(m) * h
    X = np.stack(np.meshgrid(xs, xs, indexing="xy"), axis=-1).reshape(-1, 2)
    N = m * m
    kind = np.full(N, DIRICHLET, dtype=np.uint8)
    sizes, idx, w = [], [], []
    for k in range(N):
        i, j = k % m, k // m
        if 0 < i < m - 1 and 0 < j < m - 1:
            kind[k] = INTERIOR
            sizes.append(5)
            idx += [k, k + 1, k - 1, k + m, k - m]
            w += [-4.0 / h ** 2] + [1.0 / h ** 2] * 4
        else:
            sizes.append(1)
            idx.append(k)
            w.append(0.0)
    off = ns.offsets_from_sizes(np.asarray(sizes, dtype=np.int64))
    return X, h, off, np.asarray(idx, dtype=np.int64), np.asarray(w), kind
