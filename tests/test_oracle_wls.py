"""Pins of the GWLS oracle (Sec. 2.2.1).

* polynomial reproduction: the weights are exact for every monomial of degree
  <= P (they satisfy B^T w = (L b)(0), eq. wbsys), with and without weighting;
* n = m: least squares is interpolation, so the weights are the textbook finite
  differences of tests/golden/fd_stars.txt whatever the weight function;
* the 3 x 3 lattice with the quadratic basis, derived by hand: by symmetry the fit
  reduces to the span of 1, x^2, y^2; with q_i = omega_i^2, A1 = q_c + 4 q_e + 4 q_k,
  A2 = 2 q_e + 4 q_k, A3 = 4 q_k (centre, edge and corner values) the Laplacian
  weight of node i is 2 q_i (r_i^2 - 2 A2 / A1) / (A2 + A3 - 2 A2^2 / A1) / h^2
  (r_i in lattice units), and the d/dx weight is q_i x_i / (sum_j q_j x_j^2) / h;
  unweighted, the Laplacian weights are (2/3, -1/3, -4/3) / h^2 at corners, edges
  and centre;
* fewer nodes than monomials: singular.
"""
import math

import numpy as np
import pytest

import nodesets as ns
from oracle import knn, wls
from test_oracle_weights import golden_stars


def _lattice3():
    return np.array([[0, 0], [1, 0], [-1, 0], [0, 1], [0, -1], [1, 1], [1, -1], [-1, 1], [-1, -1]], float)


@pytest.mark.parametrize("weight", [wls.UNIT, wls.GAUSSIAN])
def test_lattice_closed_form(weight):
    h = 0.037
    c = np.array([0.4, -1.1])
    L = _lattice3()
    Xs = c + h * L
    sigma = 0.8
    W = wls.stencil_weights(Xs, 2, ("lap", "dx", "dy"), weight=weight, sigma=sigma)
    r2 = np.sum(L * L, axis=1)
    s_lat = math.sqrt(2.0)                                    # the largest offset, in lattice units
    om = np.ones(9) if weight == wls.UNIT else np.exp(-(r2 / s_lat ** 2) / sigma ** 2)
    q = om * om
    qc, qe, qk = q[0], q[1], q[5]
    A1, A2, A3 = qc + 4 * qe + 4 * qk, 2 * qe + 4 * qk, 4 * qk
    lap = 2 * q * (r2 - 2 * A2 / A1) / (A2 + A3 - 2 * A2 * A2 / A1) / h ** 2
    dx = q * L[:, 0] / np.sum(q * L[:, 0] ** 2) / h
    dy = q * L[:, 1] / np.sum(q * L[:, 1] ** 2) / h
    np.testing.assert_allclose(W[0], lap, rtol=1e-12, atol=1e-12 / h ** 2)
    np.testing.assert_allclose(W[1], dx, rtol=1e-12, atol=1e-12 / h)
    np.testing.assert_allclose(W[2], dy, rtol=1e-12, atol=1e-12 / h)
    if weight == wls.UNIT:
        np.testing.assert_allclose(W[0] * h * h, [-4 / 3] + [-1 / 3] * 4 + [2 / 3] * 4, atol=1e-12)


@pytest.mark.parametrize("weight", [wls.UNIT, wls.GAUSSIAN])
def test_unisolvent_stars_are_finite_differences(weight):
    g = golden_stars()
    h = 0.021
    W2 = wls.stencil_weights(np.array([0.3, 0.2]) + h * g["2d.offsets"], 2, ("lap", "dx", "dy"), weight=weight)
    np.testing.assert_allclose(W2[0] * h * h, g["2d.lap_h2"], atol=1e-11)
    np.testing.assert_allclose(W2[1] * h, g["2d.dx_h"], atol=1e-11)
    np.testing.assert_allclose(W2[2] * h, g["2d.dy_h"], atol=1e-11)
    W3 = wls.stencil_weights(np.array([0.3, 0.2, -0.5]) + h * g["3d.offsets"], 2, ("lap", "dz"), weight=weight)
    np.testing.assert_allclose(W3[0] * h * h, g["3d.lap_h2"], atol=1e-11)
    np.testing.assert_allclose(W3[1] * h, g["3d.dz_h"], atol=1e-11)


@pytest.mark.parametrize("d,P,n", [(2, 2, 12), (2, 4, 30), (3, 2, 20), (3, 3, 35)])
def test_polynomial_reproduction(d, P, n):
    nd = ns.disk(0.09, 31) if d == 2 else ns.cube_minus_sphere(1.0 / 8, 32)
    ops = ("lap", "dx", "dy", "dz")[:d + 1]
    off, idx = knn.knn_exact(nd.X, n)
    W, st = wls.weights(nd.X, off, idx, P, ops, weight=wls.GAUSSIAN, sigma=1.0)
    assert np.all(st == 0)
    rng = np.random.default_rng(d * 10 + P)
    from oracle.rbffd import monomial_exponents
    E = monomial_exponents(d, P)
    coef = rng.normal(size=E.shape[0])
    X = nd.X
    u = np.zeros(nd.N)
    lap = np.zeros(nd.N)
    grads = np.zeros((d, nd.N))
    for c0, e in zip(coef, E):
        u += c0 * np.prod(X ** e, axis=1)
        for a in range(d):
            if e[a] >= 2:
                ee = e.copy()
                ee[a] -= 2
                lap += c0 * e[a] * (e[a] - 1) * np.prod(X ** ee, axis=1)
            if e[a] >= 1:
                ee = e.copy()
                ee[a] -= 1
                grads[a] += c0 * e[a] * np.prod(X ** ee, axis=1)
    row = np.repeat(np.arange(nd.N), n)
    approx = [np.bincount(row, weights=W[r] * u[idx], minlength=nd.N) for r in range(len(ops))]
    scale = np.abs(u).max() * np.abs(W).max(axis=1)
    assert np.abs(approx[0] - lap).max() <= 1e-8 * scale[0]
    for a in range(d):
        assert np.abs(approx[1 + a] - grads[a]).max() <= 1e-8 * scale[1 + a]


def test_too_few_nodes_is_singular():
    nd = ns.disk(0.2, 3)
    off, idx = knn.knn_exact(nd.X, 5)
    W, st = wls.weights(nd.X, off, idx, 2, ("lap",))
    assert np.all(st == -1) and np.all(np.isnan(W))
