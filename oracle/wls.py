"""Oracle of generalized weighted least squares weights (Sec. 2.2.1, the GWLS engine).

Test infrastructure only: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the library.

Around the centre p* the approximant is u_hat(p) = b((p - p*)/s)^T alpha with b
the monomials of total degree <= P (the standard WLS choice of basis);
alpha minimises ||W (B alpha - u)||_2 with B_ij = b_j((p_i - p*)/s) and
W = diag(omega((p_i - p*)/s)).  Applying L to u_hat gives the weights in closed
form with the Moore-Penrose pseudo-inverse:

    w^T = (L b)(0)^T (W B)^+ W,

mapped back to physical units by s^(-order).  The same weights are W y with y
the minimum-norm solution of (W B)^T y = (L b)(0), eq. (wbsys).

Readings (the paper leaves them open): omega(x) = exp(-||x||^2 / sigma^2)
(Gaussian) or omega = 1 (unweighted); s and the monomial order as for the
RBF-FD oracle (s = the largest offset; graded order); the basis is complete
only if W B has full column rank m, which needs n >= m; otherwise the stencil
is reported singular.
"""
from __future__ import annotations

import numpy as np

from .rbffd import OP_AXES, OP_AXIS, OP_ORDER, monomial_exponents, scale_factor

UNIT, GAUSSIAN = 0, 1


def weight_function(Xh: np.ndarray, kind: int, sigma: float) -> np.ndarray:
    """omega at the scaled offsets Xh [n, d]."""
    if kind == UNIT:
        return np.ones(Xh.shape[0])
    if kind == GAUSSIAN:
        return np.exp(-np.sum(Xh * Xh, axis=1) / (sigma * sigma))
    raise ValueError(kind)


def operator_of_basis(E: np.ndarray, ops) -> np.ndarray:
    """(L b)(0) for every monomial b (rows) and operator (columns), in scaled units."""
    Lb = np.zeros((E.shape[0], len(ops)))
    for c, op in enumerate(ops):
        for l in range(E.shape[0]):
            if op == "lap":
                Lb[l, c] = 2.0 if (E[l].sum() == 2 and E[l].max() == 2) else 0.0
            elif op in OP_AXES:
                a, b = OP_AXES[op]
                e = np.zeros(E.shape[1], dtype=np.int64)
                e[a] += 1
                e[b] += 1
                Lb[l, c] = (2.0 if a == b else 1.0) if np.array_equal(E[l], e) else 0.0
            else:
                Lb[l, c] = 1.0 if (E[l].sum() == 1 and E[l, OP_AXIS[op]] == 1) else 0.0
    return Lb


def stencil_weights(Xs, P: int, ops=("lap",), weight: int = GAUSSIAN, sigma: float = 1.0, scale: str = "max"):
    """Weights of one stencil (centre first): [R, n], or None when W B is rank deficient."""
    Xs = np.asarray(Xs, dtype=np.float64)
    n, d = Xs.shape
    O = Xs - Xs[0]
    s = float(scale_factor(O[None], scale)[0])
    Xh = O / s
    E = monomial_exponents(d, P)
    B = np.ones((n, E.shape[0]))
    for l in range(E.shape[0]):
        for a in range(d):
            B[:, l] *= Xh[:, a] ** E[l, a]
    om = weight_function(Xh, weight, sigma)
    WB = om[:, None] * B
    if n < E.shape[0] or np.linalg.matrix_rank(WB) < E.shape[0]:
        return None
    Lb = operator_of_basis(E, ops)
    Wt = (Lb.T @ np.linalg.pinv(WB)) * om[None, :]          # (L b)^T (W B)^+ W
    for c, op in enumerate(ops):
        Wt[c] /= s ** OP_ORDER[op]
    return Wt


def weights(X, offsets, idx, P: int, ops=("lap",), weight: int = GAUSSIAN, sigma: float = 1.0,
            scale: str = "max"):
    """(W [R, nnz], status [N]): status -1 and NaN weights for rank-deficient stencils."""
    X = np.asarray(X, dtype=np.float64)
    offsets = np.asarray(offsets, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    N = offsets.shape[0] - 1
    W = np.full((len(ops), int(offsets[-1])), np.nan)
    status = np.zeros(N, dtype=np.int8)
    for i in range(N):
        a, b = offsets[i], offsets[i + 1]
        Wi = stencil_weights(X[idx[a:b]], P, ops, weight, sigma, scale)
        if Wi is None:
            status[i] = -1
        else:
            W[:, a:b] = Wi
    return W, status
