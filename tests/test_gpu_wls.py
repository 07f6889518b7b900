"""GPU GWLS weights (Sec. 2.2.1) against the oracle.

Both sides take the same stencils (the oracle's own exact kNN) and compute
w^T = (L b)(0)^T (W B)^+ W in float64 (GPU: Householder QR; oracle: the
pseudo-inverse).  Bar: the scaled error max |w_gpu - w_oracle| h^ord /
max(1, max |w_oracle| h^ord) <= 1e-10 per stencil, as for the FP64 RBF-FD
weights; statuses equal.
"""
import numpy as np
import pytest
import torch

import nodesets as ns
from oracle import knn, wls

pytestmark = pytest.mark.gpu
ORD = {"lap": 2, "dx": 1, "dy": 1, "dz": 1}


def _rb():
    import paper_1912_13282_amd as rb
    return rb


def _scaled_err(wg, wo, ops, off, h):
    hn = np.repeat(h, np.diff(off))
    worst = 0.0
    for c, op in enumerate(ops):
        sc = hn ** ORD[op]
        den = max(1.0, float(np.nanmax(np.abs(wo[c]) * sc)))
        worst = max(worst, float(np.nanmax(np.abs(wg[c] - wo[c]) * sc)) / den)
    return worst


# d, degree, n, weight, scale_mode, sigma.  kappa(W B) over the stencils stays below 3e4 in every
# case (measured with the oracle), where both float64 routes agree far inside the bar; a Gaussian
# of width 0.7 on offsets scaled by the closest distance (up to 4) would push kappa to 2e8.
CASES = [
    (2, 2, 12, "gaussian", 0, 0.7), (2, 2, 12, "unit", 1, 1.0), (2, 4, 30, "gaussian", 0, 0.7),
    (2, 3, 64, "unit", 0, 1.0), (3, 2, 20, "gaussian", 0, 0.7), (3, 3, 35, "gaussian", 1, 3.0),
    (3, 4, 50, "unit", 0, 1.0), (3, 1, 7, "gaussian", 0, 0.7),
]


@pytest.mark.parametrize("d,P,n,weight,scale_mode,sigma", CASES)
def test_wls_parity(gpu, d, P, n, weight, scale_mode, sigma):
    rb = _rb()
    nd = ns.disk(0.05, 41) if d == 2 else ns.cube_minus_sphere(1.0 / 12, 42)
    ops = ("lap", "dx", "dy", "dz")[:d + 1]
    off, idx = knn.knn_exact(nd.X, n)
    Wo, so = wls.weights(nd.X, off, idx, P, ops, weight=wls.GAUSSIAN if weight == "gaussian" else wls.UNIT,
                         sigma=sigma, scale="max" if scale_mode == 0 else "closest")
    X = torch.from_numpy(nd.X).to(gpu)
    w, st = rb.compute_weights_wls(X, torch.from_numpy(off).to(gpu), torch.from_numpy(idx.astype(np.int32)).to(gpu),
                                   n, P, ops, weight=weight, sigma=sigma, scale_mode=scale_mode)
    wg, sg = w.cpu().numpy(), st.cpu().numpy()
    assert np.array_equal(sg, so)
    assert _scaled_err(wg, Wo, ops, off, nd.h) <= 1e-10
    w2, _ = rb.compute_weights_wls(X, torch.from_numpy(off).to(gpu), torch.from_numpy(idx.astype(np.int32)).to(gpu),
                                   n, P, ops, weight=weight, sigma=sigma, scale_mode=scale_mode)
    assert torch.equal(w, w2)


def test_wls_statuses(gpu):
    rb = _rb()
    nd = ns.disk(0.1, 43)
    N = nd.N
    sizes = np.full(N, 10, dtype=np.int64)
    sizes[[3, 7]] = 4            # fewer nodes than the 6 monomials of degree 2: singular
    off = ns.offsets_from_sizes(sizes)
    _, idx = knn.knn_exact(nd.X, sizes)
    idx = idx.astype(np.int32)
    idx[off[11] + 2] = N          # index out of range: BADSIZE
    X = torch.from_numpy(nd.X).to(gpu)
    w, st = rb.compute_weights_wls(X, torch.from_numpy(off).to(gpu), torch.from_numpy(idx).to(gpu), 10, 2,
                                   ("lap", "dx"))
    sg, wg = st.cpu().numpy(), w.cpu().numpy()
    assert sg[3] == rb.ST_SINGULAR and sg[7] == rb.ST_SINGULAR and sg[11] == rb.ST_BADSIZE
    for i in (3, 7, 11):
        assert np.all(np.isnan(wg[:, off[i]:off[i + 1]]))
    good = np.setdiff1d(np.arange(N), [3, 7, 11])
    assert np.all(sg[good] == rb.ST_OK)
    # larger stencils than n_max and than a wavefront
    with pytest.raises(rb.RbfError):
        rb.compute_weights_wls(X, torch.from_numpy(off).to(gpu), torch.from_numpy(idx).to(gpu), 65, 2, ("lap",))
    with pytest.raises(rb.RbfError):
        rb.compute_weights_wls(X, torch.from_numpy(off).to(gpu), torch.from_numpy(idx).to(gpu), 10, 2, ("lap",),
                               weight="gaussian", sigma=0.0)


def test_wls_full_size_sampled(gpu):
    """The 1,096,553-node cube minus sphere, n = 35, degree 3, four operators, Gaussian
    weight: the GPU stencils and weights of 2,000 sampled nodes against the oracle's,
    and exact derivatives of a cubic at every node."""
    rb = _rb()
    wl = ns.workload("cube_sphere3d")
    nd = wl["nodes"][0]
    N, n, P, ops = nd.N, 35, 3, ("lap", "dx", "dy", "dz")
    X = torch.from_numpy(nd.X).to(gpu)
    off = torch.arange(0, (N + 1) * n, n, dtype=torch.int64, device=gpu)
    idx = rb.select_stencils(X, off, n)
    w, st = rb.compute_weights_wls(X, off, idx, n, P, ops, weight="gaussian", sigma=1.0)
    assert int((st != 0).sum()) == 0
    sample = np.sort(np.random.default_rng(9).choice(N, 2000, replace=False))
    soff, sidx = knn.knn_exact(nd.X, n, nodes=sample)
    pos = (sample[:, None] * n + np.arange(n)).reshape(-1)
    assert np.array_equal(idx.cpu().numpy()[pos], sidx)
    Wo = np.concatenate([wls.stencil_weights(nd.X[sidx[soff[i]:soff[i + 1]]], P, ops, wls.GAUSSIAN, 1.0)
                         for i in range(sample.size)], axis=1)
    wg = w[:, torch.from_numpy(pos).to(gpu)].cpu().numpy()
    assert _scaled_err(wg, Wo, ops, soff, nd.h[sample]) <= 1e-10
    # exact for a cubic (the basis), at every node
    x, y, z = (X[:, a] for a in range(3))
    u = x ** 3 - 2 * x * y * z + 0.5 * y * y * z + z
    lap = 6 * x + z
    dx = 3 * x * x - 2 * y * z
    out = rb.apply_operators(off, idx, w, n, u)
    scale = w.abs().amax(dim=1) * u.abs().max()
    assert float((out[0] - lap).abs().max() / scale[0]) < 1e-9
    assert float((out[1] - dx).abs().max() / scale[1]) < 1e-9
