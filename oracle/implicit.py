"""Oracle of the implicit system M u = r (Sec. 2.3.2, eqs. implicit-start..implicit-end).

Test infrastructure only: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the library.

For L u = f in the domain, u = g_d on Dirichlet nodes and du/dn = g_n on
Neumann nodes, row i of M is
    interior:  M[i, I_ij] = (w_L)_j,                          r_i = f(p_i)
    Dirichlet: M[i, i] = 1,                                   r_i = g_d(p_i)
    Neumann:   M[i, I_ij] = sum_l n_l (w_{d_l})_j,            r_i = g_n(p_i)
The values are returned in the stencil layout (one value per stencil entry; a
Dirichlet row holds 1 at the node itself and 0 at the other entries), and the
solution of M u = r is the direct sparse solve.
"""
from __future__ import annotations

import numpy as np

INTERIOR, DIRICHLET, NEUMANN = 0, 1, 2


def assemble(offsets, idx, w_lap, w_grad, kind, normals, f=None, g=None):
    """(vals [nnz], rhs [N]) of M u = r in the stencil layout."""
    offsets = np.asarray(offsets, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    N = offsets.shape[0] - 1
    vals = np.empty(int(offsets[-1]))
    rhs = np.empty(N)
    for i in range(N):
        a, b = offsets[i], offsets[i + 1]
        if kind[i] == INTERIOR:
            vals[a:b] = w_lap[a:b]
            rhs[i] = 0.0 if f is None else f[i]
        elif kind[i] == DIRICHLET:
            assert idx[a] == i, "the first stencil node is the node itself"
            vals[a:b] = 0.0
            vals[a] = 1.0
            rhs[i] = 0.0 if g is None else g[i]
        elif kind[i] == NEUMANN:
            assert idx[a] == i, "the first stencil node is the node itself"
            vals[a:b] = np.asarray(normals[i]) @ np.asarray(w_grad)[:, a:b]
            rhs[i] = 0.0 if g is None else g[i]
        else:
            raise ValueError(f"node kind {kind[i]}")
    return vals, rhs


def matrix(offsets, idx, vals, N=None):
    """The scipy CSR matrix of a stencil-layout system (duplicate entries add up)."""
    import scipy.sparse as sp

    offsets = np.asarray(offsets, dtype=np.int64)
    N = offsets.shape[0] - 1 if N is None else N
    row = np.repeat(np.arange(offsets.shape[0] - 1), np.diff(offsets))
    return sp.csr_matrix((np.asarray(vals), (row, np.asarray(idx, dtype=np.int64))), shape=(N, N))


def solve(offsets, idx, vals, rhs):
    """u with M u = r, by a sparse LU factorisation."""
    import scipy.sparse.linalg as spla

    return spla.spsolve(matrix(offsets, idx, vals).tocsc(), np.asarray(rhs))
