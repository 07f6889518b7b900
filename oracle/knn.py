"""Oracle stencil selection (Sec. 2.1; FindClosest of Sec. 3.1).  Test infrastructure only.

Definition.  Node i's stencil is I(i) = (i, j_1, ..., j_{n_i - 1}) where the j's
are the n_i - 1 nodes j != i with the smallest key, ties broken by the smaller
index.  The node itself is always first (Sec. 2.1 assumes I_{i,1} = i).

Reading of the paper (the metric is not stated): Euclidean distance, compared
through the FP64 key ((dx*dx + dy*dy) + dz*dz) with dx = x_j - x_i, every
operation correctly rounded and no fused multiply-add.  NumPy evaluates each of
these array operations separately, which is exactly that rounding sequence.
"""
from __future__ import annotations

import numpy as np


def sq_key(X: np.ndarray, i: int, J: np.ndarray) -> np.ndarray:
    """FP64 keys of nodes J relative to node i, left-to-right sum of squares."""
    D = X[J] - X[i]
    k = D[:, 0] * D[:, 0]
    for a in range(1, X.shape[1]):
        k = k + D[:, a] * D[:, a]
    return k


def knn_bruteforce(X: np.ndarray, sizes) -> tuple[np.ndarray, np.ndarray]:
    """O(N^2) stencils.  Returns (offsets[N+1] int64, idx[nnz] int32)."""
    X = np.asarray(X, dtype=np.float64)
    N = X.shape[0]
    sizes = np.broadcast_to(np.asarray(sizes, dtype=np.int64), (N,))
    off = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    idx = np.empty(off[-1], dtype=np.int32)
    allj = np.arange(N)
    for i in range(N):
        J = np.delete(allj, i)
        k = sq_key(X, i, J)
        order = np.lexsort((J, k))          # primary: key, secondary: index
        idx[off[i]] = i
        idx[off[i] + 1:off[i + 1]] = J[order[:sizes[i] - 1]]
    return off, idx


def knn_exact(X: np.ndarray, sizes, chunk: int = 65536, extra: int = 8, nodes=None):
    """Same result as knn_bruteforce for large N.

    With ``nodes`` given, only those nodes' stencils are computed (against all N
    nodes); offsets and idx then cover the listed nodes in order.

    A k-d tree (SciPy) proposes k' candidates per node; the exact FP64 keys of
    the candidates are re-ranked by (key, index).  The selection is exact when
    the last selected key is below the squared distance of the k'-th tree
    candidate by a relative margin of 1e-9 (every node not proposed is at least
    that far away); otherwise the node is queried again with k' doubled.
    """
    from scipy.spatial import cKDTree

    X = np.asarray(X, dtype=np.float64)
    N, d = X.shape
    sizes = np.broadcast_to(np.asarray(sizes, dtype=np.int64), (N,))
    nodes = np.arange(N) if nodes is None else np.asarray(nodes, dtype=np.int64)
    slot = np.full(N, -1, dtype=np.int64)          # position of a node in the output
    slot[nodes] = np.arange(nodes.size)
    off = np.zeros(nodes.size + 1, dtype=np.int64)
    np.cumsum(sizes[nodes], out=off[1:])
    idx = np.empty(off[-1], dtype=np.int32)
    tree = cKDTree(X)
    nmax = int(sizes[nodes].max())

    pending = nodes.copy()
    kq = nmax + extra
    while pending.size:
        kq_eff = min(kq, N)
        redo = []
        for s in range(0, pending.size, chunk):
            Q = pending[s:s + chunk]
            dist, J = tree.query(X[Q], k=kq_eff)
            J = J.reshape(len(Q), -1)
            dist = dist.reshape(len(Q), -1)
            D = X[J] - X[Q][:, None, :]
            K = D[..., 0] * D[..., 0]
            for a in range(1, d):
                K = K + D[..., a] * D[..., a]
            K = np.where(J == Q[:, None], np.inf, K)      # the node itself is placed first
            order = np.lexsort((J, K), axis=-1)
            Js = np.take_along_axis(J, order, axis=-1)
            Ks = np.take_along_axis(K, order, axis=-1)
            ni = sizes[Q]
            rr = np.arange(len(Q))
            last = Ks[rr, np.maximum(ni - 2, 0)]
            ok = (ni == 1) | (kq_eff >= N) | (np.isfinite(last) & (last < dist[:, -1] ** 2 * (1.0 - 1e-9)))
            redo.append(Q[~ok])
            for nv in np.unique(ni[ok]):
                rows = np.nonzero(ok & (ni == nv))[0]
                base = off[slot[Q[rows]]]
                idx[base] = Q[rows]
                if nv > 1:
                    pos = base[:, None] + np.arange(1, nv)[None, :]
                    idx[pos] = Js[rows, :nv - 1]
        pending = np.concatenate(redo).astype(np.int64) if redo else np.zeros(0, np.int64)
        kq *= 2
    return off, idx
