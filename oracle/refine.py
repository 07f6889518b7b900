"""Oracle for the mixed-precision solve: FP32 LU + FP64-residual iterative refinement.

Test infrastructure only.  The paper solves eq. (rbf-system-aug) by LU in
double precision; this emulation predicts which stencils a mixed-precision
solve accepts and which it must send back to the plain FP64 solve.

Steps (classical mixed-precision refinement; the stopping test is the one of
LAPACK dsgesv):
    factor K in float32 (LAPACK sgetrf, partial pivoting);
    x_0 = float32 solve of K x = b, promoted to float64;
    for t = 0, 1, ...:
        r_t = b - K x_t in float64;
        accept if t >= 1 and every column c has
            max|r_t[:, c]| <= sqrt(M) * 2^-53 * ||K||_inf * max|x_t[:, c]|;
        reject (fall back to float64 LU) if t == max_iters;
        x_{t+1} = x_t + float32 solve of K d = r_t.
With max_iters = 0 nothing is accepted.
"""
from __future__ import annotations

import numpy as np


def ir_solve(K: np.ndarray, B: np.ndarray, max_iters: int = 10):
    """Returns (x float64 [M, R], corrections used, accepted)."""
    from scipy.linalg import lu_factor, lu_solve

    K = np.asarray(K, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64).reshape(K.shape[0], -1)
    M = K.shape[0]
    lu32 = lu_factor(K.astype(np.float32), check_finite=False)
    x = lu_solve(lu32, B.astype(np.float32)).astype(np.float64)
    anrm = np.abs(K).sum(axis=1).max()
    tol = np.sqrt(M) * 2.0 ** -53 * anrm
    for t in range(max_iters + 1):
        r = B - K @ x
        if t >= 1 and np.all(np.abs(r).max(axis=0) <= tol * np.abs(x).max(axis=0)):
            return x, t, True
        if t == max_iters:
            break
        x = x + lu_solve(lu32, r.astype(np.float32)).astype(np.float64)
    return x, max_iters, False
