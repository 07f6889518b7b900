"""Oracle of the general second-order operator built from stored weights, eq. (gen-op), Sec. 3.3.

Test infrastructure only: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the library.

For L = sum_alpha a_alpha(p) d^alpha the weights at node i are
w_{L,p_i} = sum_alpha a_alpha(p_i) w_{d^alpha, p_i}: a per-node linear
combination of the stored operator weights.
"""
from __future__ import annotations

import numpy as np


def combine(offsets, W, coef):
    """out[p] = sum_k coef[i][k] W[k][p] for the positions p of stencil i.
    W [K, nnz] (operator-major), coef [N, K]."""
    offsets = np.asarray(offsets, dtype=np.int64)
    W = np.atleast_2d(np.asarray(W, dtype=np.float64))
    coef = np.asarray(coef, dtype=np.float64).reshape(offsets.shape[0] - 1, W.shape[0])
    out = np.empty(W.shape[1])
    for i in range(offsets.shape[0] - 1):
        a, b = offsets[i], offsets[i + 1]
        out[a:b] = coef[i] @ W[:, a:b]
    return out
