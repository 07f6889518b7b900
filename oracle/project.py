"""Oracle projection of surrogate weights onto the reproduction constraints.

Test infrastructure only.  The second block row of eq. (rbf-system-aug),
Q^T w = l_q, is the polynomial-reproduction condition every RBF-FD weight
vector satisfies.  A learned weight vector y is replaced by the Euclidean-
nearest vector that satisfies it:

    w = y + Q (Q^T Q)^{-1} (l_q - Q^T y)

all in float64 (scaled coordinates).  The residual
rho = ||Q^T w - l_q||_inf / max(1, ||l_q||_inf) decides acceptance: rho > 1e-6
sends the stencil to the plain solve.
"""
from __future__ import annotations

import numpy as np

from .rbffd import monomial_exponents


def q_matrix(Xh: np.ndarray, P: int) -> np.ndarray:
    """Q [B, n, m] of scaled offsets Xh [B, n, d]."""
    B, n, d = Xh.shape
    E = monomial_exponents(d, P)
    Q = np.ones((B, n, E.shape[0]))
    for l in range(E.shape[0]):
        for a in range(d):
            Q[:, :, l] *= Xh[:, :, a] ** E[l, a]
    return Q


def lap_lq(d: int, P: int) -> np.ndarray:
    """(lap q_l)(0) for the graded monomial basis."""
    E = monomial_exponents(d, P)
    return np.array([2.0 if (e.sum() == 2 and e.max() == 2) else 0.0 for e in E])


def project(y: np.ndarray, Xh: np.ndarray, P: int, lq: np.ndarray):
    """Returns (w [B, n], rho [B]) for learned weights y [B, n]."""
    Q = q_matrix(Xh, P)
    Qt = np.swapaxes(Q, 1, 2)
    G = Qt @ Q
    rhs = lq[None, :] - np.einsum("bnm,bn->bm", Q, y)
    c = np.linalg.solve(G, rhs[..., None])[..., 0]
    w = y + np.einsum("bnm,bm->bn", Q, c)
    res = np.einsum("bnm,bn->bm", Q, w) - lq[None, :]
    rho = np.abs(res).max(axis=1) / max(1.0, float(np.abs(lq).max()))
    return w, rho
