"""Pins of the second-derivative operators and the general second-order operator
(eq. gen-op, Sec. 3.3) in the oracles.

* unisolvent stars: the weights of d2/dx_a dx_b are the quadratic interpolant's,
  tests/golden/fd_stars.txt (RBF-FD for r^3 and r^5, and GWLS);
* linearity: the right-hand side of the Laplacian is the sum of those of the pure
  second derivatives, so w_lap = w_xx + w_yy (+ w_zz) to rounding;
* exactness for polynomials of degree <= P, including mixed derivatives;
* the general operator sum_alpha a_alpha(p) w_alpha applied to a quadratic field
  equals the operator applied analytically.
"""
import numpy as np
import pytest

import nodesets as ns
from oracle import combine, knn, rbffd, wls
from test_oracle_weights import golden_stars

H2 = ("dxx", "dxy", "dxz", "dyy", "dyz", "dzz")


@pytest.mark.parametrize("engine", ["rbf3", "rbf5", "wls"])
def test_second_derivative_stars(engine):
    g = golden_stars()
    h = 0.017

    def weights(Xs, ops):
        if engine == "wls":
            return wls.stencil_weights(Xs, 2, ops, weight=wls.GAUSSIAN)
        return rbffd.stencil_weights(Xs, 2, ops, phs_power=3 if engine == "rbf3" else 5)
    W2 = weights(np.array([0.2, -0.4]) + h * g["2d.offsets"], ("dxx", "dxy", "dyy"))
    for c, k in enumerate(("2d.dxx_h2", "2d.dxy_h2", "2d.dyy_h2")):
        np.testing.assert_allclose(W2[c] * h * h, g[k], atol=1e-10)
    W3 = weights(np.array([0.2, -0.4, 0.9]) + h * g["3d.offsets"], ("dxz", "dyz", "dzz"))
    for c, k in enumerate(("3d.dxz_h2", "3d.dyz_h2", "3d.dzz_h2")):
        np.testing.assert_allclose(W3[c] * h * h, g[k], atol=1e-10)


@pytest.mark.parametrize("d,P,n", [(2, 2, 15), (3, 3, 35)])
def test_laplacian_is_the_trace(d, P, n):
    nd = ns.disk(0.1, 51) if d == 2 else ns.cube_minus_sphere(1.0 / 7, 52)
    off, idx = knn.knn_exact(nd.X, n)
    pure = ("dxx", "dyy", "dzz")[:d]
    W, st = rbffd.weights(nd.X, off, idx, P, ("lap",) + pure)
    assert np.all(st == 0)
    tr = W[1:].sum(axis=0)
    assert np.abs(tr - W[0]).max() <= 1e-9 * np.abs(W[0]).max()


@pytest.mark.parametrize("engine", ["rbf", "wls"])
def test_second_derivatives_exact_for_polynomials(engine):
    nd = ns.cube_minus_sphere(1.0 / 7, 53)
    n, P = 35, 3
    off, idx = knn.knn_exact(nd.X, n)
    if engine == "rbf":
        W, st = rbffd.weights(nd.X, off, idx, P, H2)
    else:
        W, st = wls.weights(nd.X, off, idx, P, H2)
    assert np.all(st == 0)
    x, y, z = nd.X.T
    u = x ** 3 - 2 * x * y * z + 0.5 * y * y * z + 3 * x * z * z - y ** 3 + x * y
    exact = {"dxx": 6 * x, "dxy": -2 * z + 1, "dxz": -2 * y + 6 * z, "dyy": z - 6 * y, "dyz": -2 * x + y,
             "dzz": 6 * x}
    row = np.repeat(np.arange(nd.N), n)
    for c, op in enumerate(H2):
        approx = np.bincount(row, weights=W[c] * u[idx], minlength=nd.N)
        assert np.abs(approx - exact[op]).max() <= 1e-8 * np.abs(W[c]).max() * np.abs(u).max(), op


def test_general_operator_of_stored_weights():
    """L = a(p) d_xx + b(p) d_xy + c(p) d_y with coefficients varying per node, applied
    to a quadratic (exact for degree-2 augmentation)."""
    nd = ns.disk(0.08, 54)
    n = 15
    off, idx = knn.knn_exact(nd.X, n)
    ops = ("dy", "dxx", "dxy")
    W, st = rbffd.weights(nd.X, off, idx, 2, ops)
    x, y = nd.X.T
    coef = np.stack([np.cos(x), 1 + x * y, np.exp(y)], axis=1)     # [N, 3] in the order of ops
    wL = combine.combine(off, W, coef)
    u = 2 * x * x - 3 * x * y + y * y + 4 * y - 1
    Lu_exact = coef[:, 0] * (-3 * x + 2 * y + 4) + coef[:, 1] * 4.0 + coef[:, 2] * (-3.0)
    row = np.repeat(np.arange(nd.N), n)
    approx = np.bincount(row, weights=wL * u[idx], minlength=nd.N)
    assert np.abs(approx - Lu_exact).max() <= 1e-9 * np.abs(W).max() * np.abs(u).max() * 3
    # combining the pure second derivatives with unit coefficients gives the Laplacian
    W2, _ = rbffd.weights(nd.X, off, idx, 2, ("lap", "dxx", "dyy"))
    wl = combine.combine(off, W2[1:], np.ones((nd.N, 2)))
    assert np.abs(wl - W2[0]).max() <= 1e-9 * np.abs(W2[0]).max()
