"""Oracle RBF-FD weights with monomial augmentation (Sec. 2.2.2).  Test infrastructure only.

For a stencil with nodes p_1 = p* (the centre), p_2, ..., p_n the weights of an
operator L at p* solve the augmented system, eq. (rbf-system-aug):

    [ A   Q ] [ w      ]   [ l_phi ]
    [ Q^T 0 ] [ lambda ] = [ l_q   ]

A_jk = phi(||x_j - x_k||), Q_jl = q_l(x_j), l_phi_j = (L phi_j)(0),
l_q_l = (L q_l)(0), lambda is discarded.  Coordinates are shifted to p* and
scaled by s (Sec. 2.2.1, 2.2.2): x_j = (p_j - p*) / s.

Readings of the paper (it leaves these open):
* phi(r) = r^k, polyharmonic spline with odd k (k = 3 unless stated; the
  Laplacian-error study of Sec. 3.2 also uses k = 5);
* s = max_j ||p_j - p*|| (the stencil radius; "three scaling functions" are named
  but not defined); s = distance to the closest node is available as an option;
* the augmentation degree is called P here and the number of monomials
  m = C(P + d, d) (the paper writes l = binom(m + d, d) with m the degree);
* monomials are plain powers of the scaled offsets in graded order (total
  degree ascending, then x-power descending, then y-power descending); the
  weights do not depend on this order;
* the operators are built in scaled coordinates, evaluated at x = 0 and mapped
  back with s^(-order): order 2 for the Laplacian, 1 for a first derivative;
* the system is solved by LU with partial pivoting (LAPACK gesv), the solver
  the paper names.

Closed forms used for the right-hand side (phi(r) = r^k, r = ||x - x_j||):
    Laplacian: (lap phi_j)(0) = k (k + d - 2) ||x_j||^(k-2)
    d/dx_a:    (d_a phi_j)(0) = -k ||x_j||^(k-2) x_{j,a}
    d2/dx_a dx_b: (d_ab phi_j)(0) = k ||x_j||^(k-2) delta_ab + k (k-2) ||x_j||^(k-4) x_{j,a} x_{j,b}
               (0 at x_j = 0, where the second term vanishes in the limit)
    (lap q_l)(0) = 2 if q_l = x_a^2 else 0;  (d_a q_l)(0) = 1 if q_l = x_a else 0;
    (d_ab q_l)(0) = 2 if q_l = x_a^2 (a = b), 1 if q_l = x_a x_b (a != b), else 0.
The second derivatives are the operators of the general second-order
operator of eq. (gen-op), Sec. 3.3.
"""
from __future__ import annotations

import math

import numpy as np

OPS = ("lap", "dx", "dy", "dz", "dxx", "dxy", "dxz", "dyy", "dyz", "dzz")
OP_ORDER = {"lap": 2, "dx": 1, "dy": 1, "dz": 1, "dxx": 2, "dxy": 2, "dxz": 2, "dyy": 2, "dyz": 2, "dzz": 2}
OP_AXIS = {"dx": 0, "dy": 1, "dz": 2}
OP_AXES = {"dxx": (0, 0), "dxy": (0, 1), "dxz": (0, 2), "dyy": (1, 1), "dyz": (1, 2), "dzz": (2, 2)}


def monomial_exponents(d: int, P: int) -> np.ndarray:
    """Exponents alpha (|alpha| <= P) in graded order; shape [C(P+d,d), d]."""
    out = []
    for deg in range(P + 1):
        if d == 1:
            out.append((deg,))
        elif d == 2:
            for a in range(deg, -1, -1):
                out.append((a, deg - a))
        else:
            for a in range(deg, -1, -1):
                for b in range(deg - a, -1, -1):
                    out.append((a, b, deg - a - b))
    E = np.asarray(out, dtype=np.int64)
    assert E.shape[0] == math.comb(P + d, d)
    return E


def scale_factor(O: np.ndarray, scale: str = "max") -> np.ndarray:
    """s per stencil from offsets O [..., n, d] (row 0 is the centre, offset 0)."""
    r = np.sqrt(np.sum(O * O, axis=-1))
    if scale == "max":
        return r.max(axis=-1)
    if scale == "closest":
        return r[..., 1:].min(axis=-1)
    raise ValueError(scale)


def assemble(Xs: np.ndarray, P: int, ops, phs_power: int = 3, scale: str = "max"):
    """Augmented matrices and right-hand sides for a stack of stencils.

    Xs: [B, n, d] stencil node coordinates, centre first.
    Returns K [B, n+m, n+m], RHS [B, n+m, R], s [B].
    """
    Xs = np.asarray(Xs, dtype=np.float64)
    B, n, d = Xs.shape
    E = monomial_exponents(d, P)
    m = E.shape[0]
    k = phs_power
    O = Xs - Xs[:, :1, :]                       # shift to p* = p_1
    s = scale_factor(O, scale)
    Xh = O / s[:, None, None]                   # scale
    diff = Xh[:, :, None, :] - Xh[:, None, :, :]
    A = np.sqrt(np.sum(diff * diff, axis=-1)) ** k
    Q = np.ones((B, n, m))
    for l in range(m):
        for a in range(d):
            Q[:, :, l] *= Xh[:, :, a] ** E[l, a]
    K = np.zeros((B, n + m, n + m))
    K[:, :n, :n] = A
    K[:, :n, n:] = Q
    K[:, n:, :n] = np.swapaxes(Q, 1, 2)
    r = np.sqrt(np.sum(Xh * Xh, axis=-1))      # ||x_j||
    RHS = np.zeros((B, n + m, len(ops)))
    for c, op in enumerate(ops):
        if op == "lap":
            RHS[:, :n, c] = k * (k + d - 2) * r ** (k - 2)
            for l in range(m):
                if E[l].sum() == 2 and E[l].max() == 2:
                    RHS[:, n + l, c] = 2.0
        elif op in OP_AXES:
            a, b = OP_AXES[op]
            rk4 = np.zeros_like(r)                                   # r^(k-4); its term is 0 at r = 0
            np.power(r, k - 4.0, out=rk4, where=r > 0)
            RHS[:, :n, c] = k * (a == b) * r ** (k - 2) + k * (k - 2) * rk4 * Xh[:, :, a] * Xh[:, :, b]
            for l in range(m):
                e = np.zeros(d, dtype=np.int64)
                e[a] += 1
                e[b] += 1
                if np.array_equal(E[l], e):
                    RHS[:, n + l, c] = 2.0 if a == b else 1.0
        else:
            a = OP_AXIS[op]
            RHS[:, :n, c] = -k * r ** (k - 2) * Xh[:, :, a]
            for l in range(m):
                if E[l].sum() == 1 and E[l, a] == 1:
                    RHS[:, n + l, c] = 1.0
    return K, RHS, s


def stencil_weights(Xs: np.ndarray, P: int, ops=("lap",), phs_power: int = 3, scale: str = "max"):
    """Weights of one stencil.  Xs: [n, d], centre first.  Returns [R, n] float64."""
    K, RHS, s = assemble(np.asarray(Xs)[None], P, ops, phs_power, scale)
    n = Xs.shape[0]
    sol = np.linalg.solve(K[0], RHS[0])          # LAPACK gesv: LU with partial pivoting
    W = sol[:n, :].T.copy()                     # lambda (rows n..n+m-1) is discarded
    for c, op in enumerate(ops):
        W[c] /= s[0] ** OP_ORDER[op]
    return W


def weights(X, offsets, idx, P, ops=("lap",), phs_power: int = 3, scale: str = "max",
            batch: int = 4096):
    """Weights of every stencil.  Returns (W [R, nnz] float64, status [N] int8).

    P is a scalar or a per-node array.  Stencils of equal (n, P) are stacked and
    solved by the same gesv call per matrix; a singular system gives status -1 and
    NaN weights.
    """
    X = np.asarray(X, dtype=np.float64)
    offsets = np.asarray(offsets, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    N = offsets.shape[0] - 1
    sizes = np.diff(offsets)
    Pn = np.broadcast_to(np.asarray(P, dtype=np.int64), (N,))
    R = len(ops)
    W = np.full((R, offsets[-1]), np.nan)
    status = np.zeros(N, dtype=np.int8)
    keys = sizes * 16 + Pn
    for key in np.unique(keys):
        nodes = np.nonzero(keys == key)[0]
        n, p = int(key // 16), int(key % 16)
        for s0 in range(0, nodes.size, batch):
            sel = nodes[s0:s0 + batch]
            pos = offsets[sel][:, None] + np.arange(n)[None, :]
            Xs = X[idx[pos]]
            K, RHS, s = assemble(Xs, p, ops, phs_power, scale)
            try:
                sol = np.linalg.solve(K, RHS)
                good = np.ones(sel.size, dtype=bool)
            except np.linalg.LinAlgError:
                sol = np.full(RHS.shape, np.nan)
                good = np.zeros(sel.size, dtype=bool)
                for b in range(sel.size):
                    try:
                        sol[b] = np.linalg.solve(K[b], RHS[b])
                        good[b] = True
                    except np.linalg.LinAlgError:
                        pass
            good &= np.all(np.isfinite(sol), axis=(1, 2))
            for c, op in enumerate(ops):
                Wc = sol[:, :n, c] / (s[:, None] ** OP_ORDER[op])
                Wc[~good] = np.nan
                W[c, pos] = Wc
            status[sel[~good]] = -1
    return W, status


def weights_subset(X, offsets, idx, nodes, P, ops=("lap",), phs_power: int = 3, scale: str = "max"):
    """Weights of the stencils of the listed nodes only: dict node -> [R, n_i]."""
    offsets = np.asarray(offsets, dtype=np.int64)
    Pn = np.broadcast_to(np.asarray(P, dtype=np.int64), (offsets.shape[0] - 1,))
    out = {}
    for i in np.asarray(nodes).reshape(-1):
        st = np.asarray(idx[offsets[i]:offsets[i + 1]], dtype=np.int64)
        out[int(i)] = stencil_weights(np.asarray(X)[st], int(Pn[i]), ops, phs_power, scale)
    return out
