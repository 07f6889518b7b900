"""Oracle of explicit operator evaluation and the explicit Euler step (Sec. 2.3.1).

Test infrastructure only: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the library.

apply_operators: (L u)(p_i) ~ w_{L,p_i}^T u_{I(i)} = sum_j w_ij u_{I_ij}, for every
operator row of a weight array laid out operator-major over the stencils.

explicit_step, eqs. (exp-start)-(exp-end), for du/dt = L u + s: with u^k known,
    interior node:  u^{k+1}_i = u^k_i + dt (w_{L,p_i}^T u^k_{I(i)} + s_i)
    Dirichlet node: u^{k+1}_i = g_d(p_i, (k+1) dt)
    Neumann node:   u^{k+1}_i = (g_n - sum_{j>=2} u^k_{I_ij} sum_l n_l (w_{d_l})_j)
                                / sum_l n_l (w_{d_l})_1
where the Neumann form is the discretised normal derivative, eq. (neu), set equal
to g_n and solved for u_i (the first stencil node is p_i itself).  The source s
is the constant term of the heat example of Sec. 3.3.1 (du/dt = lap u + 5).
"""
from __future__ import annotations

import numpy as np

INTERIOR, DIRICHLET, NEUMANN = 0, 1, 2


def apply_operators(offsets, idx, w, u):
    """out[r][i] = sum over the stencil of node i of w[r][pos] u[idx[pos]] (float64)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    w = np.atleast_2d(np.asarray(w, dtype=np.float64))
    u = np.asarray(u, dtype=np.float64)
    N = offsets.shape[0] - 1
    out = np.zeros((w.shape[0], N))
    for i in range(N):
        a, b = offsets[i], offsets[i + 1]
        out[:, i] = w[:, a:b] @ u[idx[a:b]]
    return out


def explicit_step(offsets, idx, w_lap, w_grad, kind, normals, u, dt, g=None, s=None):
    """One explicit Euler step.  kind: INTERIOR, DIRICHLET or NEUMANN per node.

    w_grad [d][nnz] and normals [N][d] are read at Neumann nodes only.  g holds
    g_d at Dirichlet and g_n at Neumann nodes (None: keep u, zero flux); s is the
    source (None: 0)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    u = np.asarray(u, dtype=np.float64)
    N = offsets.shape[0] - 1
    out = np.empty(N)
    for i in range(N):
        a, b = offsets[i], offsets[i + 1]
        st = idx[a:b]
        if kind[i] == INTERIOR:
            src = 0.0 if s is None else s[i]
            out[i] = u[i] + dt * (float(np.dot(w_lap[a:b], u[st])) + src)
        elif kind[i] == DIRICHLET:
            out[i] = u[i] if g is None else g[i]
        elif kind[i] == NEUMANN:
            assert st[0] == i, "the first stencil node is the node itself"
            c = np.asarray(normals[i]) @ np.asarray(w_grad)[:, a:b]   # sum_l n_l (w_dl)_j for every j
            gn = 0.0 if g is None else g[i]
            out[i] = (gn - float(np.dot(u[st[1:]], c[1:]))) / c[0]
        else:
            raise ValueError(f"node kind {kind[i]}")
    return out
