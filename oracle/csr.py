"""Oracle CSR assembly of the operator matrix (Sec. 2.3.2).  Test infrastructure only.

Row i of the operator holds the weights of node i's stencil at the columns
I(i); the matrix has at most sum(n_i) nonzeros (eqs. implicit-start..end,
internal-node rows).  Layout: row_ptr = [0, cumsum(n_i)] (int64), columns of a
row in ascending order (int32), the values of every operator permuted alike.
"""
from __future__ import annotations

import numpy as np


def to_csr(offsets, idx, W):
    """(row_ptr [N+1] int64, col [nnz] int32, vals [R, nnz]) from stencils and weights."""
    offsets = np.asarray(offsets, dtype=np.int64)
    idx = np.asarray(idx)
    W = np.atleast_2d(np.asarray(W))
    N = offsets.shape[0] - 1
    row_of = np.repeat(np.arange(N), np.diff(offsets))
    order = np.lexsort((idx, row_of))        # by row, then by column within the row
    col = idx[order].astype(np.int32)
    vals = W[:, order]
    return offsets.copy(), col, vals


def to_scipy(row_ptr, col, vals_row, N):
    """One operator's CSR as a scipy.sparse matrix (for solves and products)."""
    import scipy.sparse as sp
    return sp.csr_matrix((np.asarray(vals_row), np.asarray(col), np.asarray(row_ptr)), shape=(N, N))
