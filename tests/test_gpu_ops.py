"""GPU second-derivative operators and the general second-order operator (eq. gen-op,
Sec. 3.3) against the oracle.

The right-hand-side slots of the weight kernels carry any four of LAP, DX, DY,
DZ, DXX, DXY, DXZ, DYY, DYZ, DZZ; every solver path (one row per lane, the
four-wave solver above 64 unknowns, FP32 + refinement, the batched persistent
form, GWLS) is compared with the oracle to the bars of the FP64 weights
(1e-10 scaled; 1e-9 for the refined form).
"""
import numpy as np
import pytest
import torch

import nodesets as ns
from oracle import combine, knn, rbffd, wls

pytestmark = pytest.mark.gpu
ORD = {"lap": 2, "dx": 1, "dy": 1, "dz": 1, "dxx": 2, "dxy": 2, "dxz": 2, "dyy": 2, "dyz": 2, "dzz": 2}


def _rb():
    import paper_1912_13282_amd as rb
    return rb


def _scaled_err(wg, wo, ops, off, h):
    hn = np.repeat(h, np.diff(off))
    worst = 0.0
    for c, op in enumerate(ops):
        sc = hn ** ORD[op]
        den = max(1.0, float(np.max(np.abs(wo[c]) * sc)))
        worst = max(worst, float(np.max(np.abs(wg[c] - wo[c]) * sc)) / den)
    return worst


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


CASES = {  # name: (node set, n, degree, ops)
    "disk_hessian": (lambda: ns.disk(0.05, 61), 15, 2, ("dxx", "dxy", "dyy")),
    "disk_mixed": (lambda: ns.disk(0.05, 62), 20, 3, ("lap", "dy", "dxy")),
    # four operators in 2D: a second derivative in the last slot, whose refinement
    # must be checked like the others
    "disk_four": (lambda: ns.disk(0.05, 71), 20, 3, ("lap", "dx", "dy", "dxx")),
    "cube_hessian_a": (lambda: ns.cube_minus_sphere(1.0 / 12, 63), 35, 3, ("dxx", "dxy", "dxz", "dyy")),
    "cube_hessian_b": (lambda: ns.cube_minus_sphere(1.0 / 12, 63), 35, 3, ("dz", "dyz", "dzz")),
    "cube_large": (lambda: ns.cube_minus_sphere(1.0 / 10, 64), 65, 4, ("dxy", "dzz")),   # n + m = 100
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", ["f64", "f32_ir"])
def test_second_derivative_parity(gpu, case, precision):
    rb = _rb()
    mk, n, P, ops = CASES[case]
    nd = mk()
    off, idx = knn.knn_exact(nd.X, n)
    Wo, so = rbffd.weights(nd.X, off, idx, P, ops)
    assert np.all(so == 0)
    w, st = rb.compute_weights(_t(nd.X, gpu), _t(off, gpu), _t(idx.astype(np.int32), gpu), n, P, ops,
                               precision=precision)
    sg = st.cpu().numpy()
    if precision == "f64":
        assert np.all(sg == rb.ST_OK)
    else:
        assert np.all((sg == rb.ST_REFINED) | (sg == rb.ST_FALLBACK))
    assert _scaled_err(w.cpu().numpy(), Wo, ops, off, nd.h) <= (1e-10 if precision == "f64" else 1e-9)


def test_laplacian_equals_trace_on_the_gpu(gpu):
    rb = _rb()
    nd = ns.cube_minus_sphere(1.0 / 14, 65)
    off, idx = knn.knn_exact(nd.X, 35)
    a = (_t(nd.X, gpu), _t(off, gpu), _t(idx.astype(np.int32), gpu), 35, 3)
    w1, _ = rb.compute_weights(*a, ("lap", "dxx", "dyy", "dzz"))
    tr = w1[1] + w1[2] + w1[3]
    assert float((tr - w1[0]).abs().max() / w1[0].abs().max()) < 1e-11
    # the classic operators are unchanged by the slot mapping: LAP computed alone is bit-equal
    w2, _ = rb.compute_weights(*a, ("lap",))
    assert torch.equal(w2[0], w1[0])


def test_second_derivatives_batched(gpu):
    """The persistent batched form with different second-derivative sets per domain."""
    rb = _rb()
    doms, refs = [], []
    for nd, n, P, ops in ((ns.disk(0.06, 66), 15, 2, ("dxx", "dxy", "dyy")),
                          (ns.cube_minus_sphere(1.0 / 10, 67), 30, 2, ("lap", "dxz", "dyz", "dzz"))):
        off, idx = knn.knn_exact(nd.X, n)
        Wo, _ = rbffd.weights(nd.X, off, idx, P, ops)
        doms.append(rb.Domain(_t(nd.X, gpu), _t(off, gpu), _t(idx.astype(np.int32), gpu), n, P, ops))
        refs.append((Wo, ops, off, nd.h))
    rb.compute_weights_batched(doms, precision="f64")
    for D, (Wo, ops, off, h) in zip(doms, refs):
        assert np.all(D.status.cpu().numpy() == rb.ST_OK)
        assert _scaled_err(D.w.cpu().numpy(), Wo, ops, off, h) <= 1e-10


def test_second_derivatives_wls(gpu):
    rb = _rb()
    nd = ns.cube_minus_sphere(1.0 / 12, 68)
    ops = ("dxx", "dxy", "dyz", "dzz")
    off, idx = knn.knn_exact(nd.X, 35)
    Wo, so = wls.weights(nd.X, off, idx, 3, ops, weight=wls.GAUSSIAN, sigma=0.7)
    w, st = rb.compute_weights_wls(_t(nd.X, gpu), _t(off, gpu), _t(idx.astype(np.int32), gpu), 35, 3, ops,
                                   weight="gaussian", sigma=0.7)
    assert np.array_equal(st.cpu().numpy(), so)
    assert _scaled_err(w.cpu().numpy(), Wo, ops, off, nd.h) <= 1e-10


def test_operator_limits(gpu):
    rb = _rb()
    nd = ns.disk(0.1, 69)
    off, idx = knn.knn_exact(nd.X, 12)
    a = (_t(nd.X, gpu), _t(off, gpu), _t(idx.astype(np.int32), gpu), 12, 2)
    with pytest.raises(rb.RbfError):
        rb.compute_weights(*a, ("lap", "dx", "dy", "dxx", "dyy"))      # five operators
    with pytest.raises(rb.RbfError):
        rb.compute_weights(*a, ("dxz",))                                # z in 2D


def test_general_operator_parity_and_exactness(gpu):
    """w_L = sum_k a_k(p) w_k (eq. gen-op) against the oracle's combination, and the
    combined operator applied to a quadratic against the exact value."""
    rb = _rb()
    nd = ns.disk(0.04, 70)
    n = 15
    off, idx = knn.knn_exact(nd.X, n)
    ops = ("dx", "dy", "dxx", "dxy")
    Wo, _ = rbffd.weights(nd.X, off, idx, 2, ops)
    x, y = nd.X.T
    coef = np.stack([np.sin(y), x * x, 1 + y, np.cos(x)], axis=1)
    ref = combine.combine(off, Wo, coef)
    got = rb.combine_operators(_t(off, gpu), _t(Wo, gpu), n, _t(coef, gpu)).cpu().numpy()
    bound = 4 * np.finfo(float).eps * np.repeat(np.abs(coef).sum(axis=1), n) * np.abs(Wo).max(axis=0) * 2
    assert np.all(np.abs(got - ref) <= bound + 1e-300)
    # applied to u = 3x^2 - xy + 2y^2 + x: L u = sin(y)(6x - y + 1) + x^2 (-x + 4y) + (1 + y) 6 + cos(x)(-1)
    w, _ = rb.compute_weights(_t(nd.X, gpu), _t(off, gpu), _t(idx.astype(np.int32), gpu), n, 2, ops)
    wl = rb.combine_operators(_t(off, gpu), w, n, _t(coef, gpu))
    u = 3 * x * x - x * y + 2 * y * y + x
    Lu = np.sin(y) * (6 * x - y + 1) + x * x * (-x + 4 * y) + (1 + y) * 6 + np.cos(x) * (-1)
    approx = rb.apply_operators(_t(off, gpu), _t(idx.astype(np.int32), gpu), wl, n, _t(u, gpu)).cpu().numpy()[0]
    assert np.abs(approx - Lu).max() <= 1e-8 * np.abs(Wo).max() * np.abs(u).max() * 4
