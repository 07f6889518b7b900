"""Pins of the implicit-system oracle (Sec. 2.3.2, eqs. implicit-start..implicit-end).

The assembled system, solved directly, must reproduce known solutions:
  * the manufactured Poisson problem of Sec. 5 (u_0 = prod sin(pi x_a) on the
    annulus) with Dirichlet rows, at the paper's stated rate N^(-2/d);
  * the same problem with the inner circle carrying the exact normal
    derivative (Neumann rows), whose error must shrink with h;
  * the closed-form steady state of the heat example of Sec. 3.3.1;
and its rows must have the textbook form on a lattice (5-point Laplacian,
one-sided second-order normal derivative).
"""
import math

import numpy as np

import nodesets as ns
from oracle import implicit, knn, poisson, rbffd
import heat_cases as hc


def _mixed_poisson(h, d=2, n=30, P=3, neumann=True, seed=5):
    """Annulus problem: lap u = lap u_0, u = u_0 on the outer boundary, and on the
    inner one either du/dn = du_0/dn (normal into the hole) or u = u_0."""
    nd = ns.annulus(h, seed, d=d)
    X = nd.X
    r = np.linalg.norm(X, axis=1)
    inner = nd.is_boundary & (r < 0.75)
    kind = np.where(nd.is_boundary, hc.DIRICHLET, hc.INTERIOR).astype(np.uint8)
    if neumann:
        kind[inner] = hc.NEUMANN
    normals = np.zeros((nd.N, d))
    normals[inner] = -X[inner] / r[inner, None]
    ops = ("lap", "dx", "dy", "dz")[:d + 1]
    off, idx = knn.knn_exact(X, n)
    W, st = rbffd.weights(X, off, idx, P, ops)
    assert np.all(st == 0)
    u0 = poisson.u0(X)
    grad = np.stack([math.pi * np.cos(math.pi * X[:, a]) * np.prod(np.sin(math.pi * np.delete(X, a, axis=1)), axis=1)
                     for a in range(d)], axis=1)
    g = np.where(kind == hc.NEUMANN, np.sum(normals * grad, axis=1), u0)
    vals, rhs = implicit.assemble(off, idx, W[0], W[1:], kind, normals, f=poisson.lap_u0(X), g=g)
    u = implicit.solve(off, idx, vals, rhs)
    return nd, float(np.abs(u - u0).max())


def test_dirichlet_poisson_converges_at_the_papers_rate():
    """Sec. 5: n = 9 in 2D, degree 2; error ~ N^(-2/d) (slope -1 against N in 2D)."""
    Ns, errs = [], []
    for h in (0.04, 0.02, 0.01):
        nd, e = _mixed_poisson(h, d=2, n=9, P=2, neumann=False)
        Ns.append(nd.N)
        errs.append(e)
    slope = np.polyfit(np.log(Ns), np.log(errs), 1)[0]
    assert -1.4 < slope < -0.7, (Ns, errs, slope)


def test_neumann_poisson_error_shrinks():
    errs = [_mixed_poisson(h, d=2)[1] for h in (0.04, 0.02, 0.01)]
    assert errs[2] < errs[1] < errs[0] and errs[2] < 1e-3, errs


def test_heat_example_steady_state_by_the_implicit_system():
    errs = []
    for h in (0.1, 0.05):
        nd, kind, normals, g = hc.annulus_heat(h)
        off, idx = knn.knn_exact(nd.X, 30)
        W, _ = rbffd.weights(nd.X, off, idx, 3, ("lap", "dx", "dy"))
        vals, rhs = implicit.assemble(off, idx, W[0], W[1:], kind, normals, f=np.full(nd.N, -5.0), g=g)
        u = implicit.solve(off, idx, vals, rhs)
        errs.append(np.abs(u - hc.annulus_steady(nd.X)).max())
    assert errs[1] < errs[0] < 0.3, errs


def test_rows_on_the_lattice():
    """Interior rows copy the Laplacian weights, Dirichlet rows are identity rows and
    a Neumann row with one-sided x-weights (-3, 4, -1)/(2h) and normal -x is
    (3, -4, 1)/(2h)."""
    X, h, off, idx, w, kind = hc.lattice_5point(6)
    N = X.shape[0]
    vals, rhs = implicit.assemble(off, idx, w, None, kind, None, f=np.arange(N, dtype=float), g=-np.ones(N))
    M = implicit.matrix(off, idx, vals).toarray()
    for i in range(N):
        if kind[i] == hc.DIRICHLET:
            assert np.array_equal(M[i], np.eye(N)[i]) and rhs[i] == -1.0
        else:
            assert M[i, i] == -4.0 / h ** 2 and abs(M[i].sum()) <= 1e-12 / h ** 2 and rhs[i] == i
    off3 = np.array([0, 3, 4, 5])
    idx3 = np.array([0, 1, 2, 1, 2])
    wg = np.stack([np.array([-3.0, 4.0, -1.0, 0.0, 0.0]) / (2 * h), np.zeros(5)])
    kind3 = np.array([hc.NEUMANN, hc.DIRICHLET, hc.DIRICHLET], dtype=np.uint8)
    nrm = np.array([[-1.0, 0.0], [0.0, 0.0], [0.0, 0.0]])
    v3, r3 = implicit.assemble(off3, idx3, np.zeros(5), wg, kind3, nrm, g=np.array([0.25, 1.0, 2.0]))
    np.testing.assert_allclose(v3[:3], np.array([3.0, -4.0, 1.0]) / (2 * h), rtol=1e-15)
    assert list(r3) == [0.25, 1.0, 2.0]
