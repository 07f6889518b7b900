"""Oracle end-to-end checks: manufactured Poisson problem and Laplacian error.

Test infrastructure only.

* Sec. 5 benchmark problem: -lap u = f in the annulus B(0,1) minus B(0,1/2),
  u = u_0 on the boundary, u_0(x) = prod_a sin(pi x_a), f = -lap u_0 = d pi^2 u_0.
  (The printed equation drops the square of the Laplacian; f = -lap u_0 fixes it.)
  The implicit system of Sec. 2.3.2: interior rows hold the Laplacian weights at
  the stencil columns with right-hand side lap u = -f; Dirichlet rows are identity
  rows with right-hand side u_0.  Solved by a sparse direct solve.
* Sec. 3.2 error of the Laplacian approximation:
  e_h = max_i | w_i^T u_I(i) - (lap u)(p_i) |, u = sin(pi x) sin(pi y).
"""
from __future__ import annotations

import math

import numpy as np


def u0(X):
    return np.prod(np.sin(math.pi * np.asarray(X)), axis=1)


def lap_u0(X):
    d = np.asarray(X).shape[1]
    return -d * math.pi ** 2 * u0(X)


def lap_error(X, offsets, idx, w_lap, u=u0, lap_u=lap_u0):
    """e_h = max over nodes of |sum_j w_j u(p_j) - lap u(p_i)|."""
    X = np.asarray(X)
    offsets = np.asarray(offsets, dtype=np.int64)
    N = offsets.shape[0] - 1
    uv = u(X)
    row = np.repeat(np.arange(N), np.diff(offsets))
    approx = np.bincount(row, weights=np.asarray(w_lap) * uv[np.asarray(idx)], minlength=N)
    return float(np.abs(approx - lap_u(X)).max())


def solve_dirichlet(X, is_boundary, offsets, idx, w_lap):
    """Solve the manufactured problem; returns (u, max |u - u_0|)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    X = np.asarray(X)
    N = X.shape[0]
    offsets = np.asarray(offsets, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    sizes = np.diff(offsets)
    row = np.repeat(np.arange(N), sizes)
    interior = ~np.asarray(is_boundary)
    keep = interior[row]
    rows = np.concatenate([row[keep], np.nonzero(~interior)[0]])
    cols = np.concatenate([idx[keep], np.nonzero(~interior)[0]])
    vals = np.concatenate([np.asarray(w_lap)[keep], np.ones(int((~interior).sum()))])
    M = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    ex = u0(X)
    rhs = np.where(interior, lap_u0(X), ex)
    u = spla.spsolve(M.tocsc(), rhs)
    return u, float(np.abs(u - ex).max())
