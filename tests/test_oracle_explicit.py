"""Pins of the explicit-evaluation oracle (Sec. 2.3.1, eqs. exp-start..exp-end, neu).

apply_operators is pinned by polynomial reproduction (the weights of degree-P
augmentation give the exact derivatives of every polynomial of degree <= P);
explicit_step by the textbook 5-point forward-time central-space update on a
lattice, its exact decay of a discrete eigenmode over many steps, the one-sided
second-order Neumann closed form, and the steady states of the heat example of
Sec. 3.3.1 (closed forms on the annulus) as fixed points.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import nodesets as ns
from oracle import explicit, knn, rbffd
import heat_cases as hc

EPS = np.finfo(np.float64).eps


def _poly_cases(d):
    """(u, lap u, grad u) of quadratic and cubic polynomials."""
    def quad(X):
        x, y = X[:, 0], X[:, 1]
        z = X[:, 2] if d == 3 else 0 * x
        u = 1.5 - 0.7 * x + 0.3 * y + 2.0 * x * x - 1.1 * x * y + 0.4 * y * y + 0.9 * z * z - 0.2 * y * z
        lap = 4.0 + 0.8 + (1.8 if d == 3 else 0.0)
        gx = -0.7 + 4.0 * x - 1.1 * y
        gy = 0.3 - 1.1 * x + 0.8 * y - 0.2 * z
        gz = 1.8 * z - 0.2 * y
        return u, np.full(X.shape[0], lap), [gx, gy, gz][:d]

    def cubic(X):
        x, y = X[:, 0], X[:, 1]
        z = X[:, 2] if d == 3 else 0 * x
        u = x ** 3 - 2.0 * x * y * y + 0.5 * z ** 3 + x * y * z
        lap = 6.0 * x - 4.0 * x + (3.0 * z if d == 3 else 0.0)
        gx = 3.0 * x * x - 2.0 * y * y + y * z
        gy = -4.0 * x * y + x * z
        gz = 1.5 * z * z + x * y
        return u, lap, [gx, gy, gz][:d]
    return quad, cubic


@pytest.mark.parametrize("d,P,n", [(2, 2, 15), (3, 3, 35)])
def test_apply_reproduces_polynomial_derivatives(d, P, n):
    nd = ns.disk(0.08, 21) if d == 2 else ns.cube_minus_sphere(1.0 / 9, 22)
    ops = ("lap", "dx", "dy", "dz")[:d + 1]
    off, idx = knn.knn_exact(nd.X, n)
    W, st = rbffd.weights(nd.X, off, idx, P, ops)
    assert np.all(st == 0)
    cases = _poly_cases(d)
    for f in cases[:1] if P == 2 else cases:
        u, lap, grad = f(nd.X)
        out = explicit.apply_operators(off, idx, W, u)
        assert out.shape == (len(ops), nd.N)
        # rounding of the dot product and of the weights scaled by h^-ord
        scale = np.abs(u).max() * np.abs(W).reshape(len(ops), -1).max(axis=1)
        np.testing.assert_allclose(out[0], lap, atol=1e-8 * scale[0], rtol=0)
        for a in range(d):
            np.testing.assert_allclose(out[1 + a], grad[a], atol=1e-8 * scale[1 + a], rtol=0)


def test_apply_ragged_rows_and_empty_row():
    # node 0 sums three entries, node 1 none, node 2 one entry that repeats an index
    off = np.array([0, 3, 3, 5])
    idx = np.array([0, 2, 1, 2, 2])
    w = np.array([[1.0, 2.0, 3.0, 0.5, 0.25], [0.0, 1.0, 0.0, 1.0, -1.0]])
    u = np.array([10.0, 20.0, 30.0])
    out = explicit.apply_operators(off, idx, w, u)
    assert np.array_equal(out, [[10.0 + 60.0 + 60.0, 0.0, 0.75 * 30.0], [30.0, 0.0, 0.0]])


def test_explicit_interior_is_ftcs_on_the_lattice():
    X, h, off, idx, w, kind = hc.lattice_5point(17)
    m = 17
    rng = np.random.default_rng(5)
    u = rng.normal(size=m * m)
    g = rng.normal(size=m * m)
    s = rng.normal(size=m * m)
    dt = 0.2 * h * h
    out = explicit.explicit_step(off, idx, w, None, kind, None, u, dt, g=g, s=s)
    U, S, G = u.reshape(m, m), s.reshape(m, m), g.reshape(m, m)
    ref = G.copy()
    ref[1:-1, 1:-1] = U[1:-1, 1:-1] + dt * ((U[1:-1, 2:] + U[1:-1, :-2] + U[2:, 1:-1] + U[:-2, 1:-1]
                                             - 4.0 * U[1:-1, 1:-1]) / h ** 2 + S[1:-1, 1:-1])
    np.testing.assert_allclose(out, ref.reshape(-1), rtol=0, atol=1e-13 * np.abs(U).max())
    # Dirichlet without g keeps u
    out2 = explicit.explicit_step(off, idx, w, None, kind, None, u, dt)
    assert np.array_equal(out2[kind == hc.DIRICHLET], u[kind == hc.DIRICHLET])


def test_explicit_eigenmode_decays_exactly():
    """sin(pi x) sin(pi y) is an eigenvector of the 5-point Laplacian with zero
    boundary values: K explicit steps multiply it by (1 + dt lambda_h)^K."""
    m = 33
    X, h, off, idx, w, kind = hc.lattice_5point(m)
    u = np.sin(math.pi * X[:, 0]) * np.sin(math.pi * X[:, 1])
    u[kind == hc.DIRICHLET] = 0.0
    lam = -(8.0 / h ** 2) * math.sin(math.pi * h / 2) ** 2
    dt = 0.2 * h * h
    K = 50
    v = u.copy()
    for _ in range(K):
        v = explicit.explicit_step(off, idx, w, None, kind, None, v, dt, g=np.zeros(m * m))
    np.testing.assert_allclose(v, (1.0 + dt * lam) ** K * u, rtol=0, atol=1e-12)


def test_explicit_neumann_one_sided_closed_form():
    """d/dx by the one-sided second-order formula (-3 u_0 + 4 u_1 - u_2)/(2h) at x = 0,
    outward normal -x: equating -du/dx to g gives u_0 = (2 h g + 4 u_1 - u_2) / 3."""
    h = 0.1
    X = np.array([[0.0, 0.0], [h, 0.0], [2 * h, 0.0]])
    off = np.array([0, 3, 4, 5])
    idx = np.array([0, 1, 2, 1, 2])
    w_dx = np.array([-3.0, 4.0, -1.0, 0.0, 0.0]) / (2 * h)
    w_dy = np.zeros(5)
    kind = np.array([hc.NEUMANN, hc.DIRICHLET, hc.DIRICHLET], dtype=np.uint8)
    normals = np.array([[-1.0, 0.0], [0.0, 0.0], [0.0, 0.0]])
    u = np.array([7.0, 1.25, -0.5])
    g = np.array([0.3, 0.0, 0.0])
    out = explicit.explicit_step(off, idx, np.zeros(5), np.stack([w_dx, w_dy]), kind, normals, u, 0.01, g=g)
    assert out[0] == pytest.approx((2 * h * g[0] + 4 * u[1] - u[2]) / 3, abs=1e-14)
    assert X.shape[0] == out.shape[0]


def _steady_system(nd, off, idx, W, kind, normals, g, s):
    """The equations a fixed point of the explicit step satisfies, as one sparse
    system: interior L u = -s, Dirichlet u = g, Neumann (normal . grad) u = g."""
    N = nd.N
    row = np.repeat(np.arange(N), np.diff(off))
    vals = W[0].copy()
    neu = kind[row] == hc.NEUMANN
    vals[neu] = (normals[row[neu], 0] * W[1][neu] + normals[row[neu], 1] * W[2][neu])
    keep = kind[row] != hc.DIRICHLET
    A = sp.csr_matrix((vals[keep], (row[keep], idx[keep])), shape=(N, N)).tolil()
    dn = np.where(kind == hc.DIRICHLET)[0]
    A[dn, dn] = 1.0
    rhs = np.where(kind == hc.INTERIOR, -s, g)
    return spl.spsolve(A.tocsr(), rhs)


@pytest.mark.parametrize("neumann_inner", [True, False])
def test_heat_example_steady_state_is_a_fixed_point(neumann_inner):
    """Heat example of Sec. 3.3.1: the discrete steady state approaches the closed
    form as h shrinks, and one explicit step leaves it unchanged."""
    errs = []
    for h in (0.1, 0.05):
        nd, kind, normals, g = hc.annulus_heat(h, neumann_inner=neumann_inner)
        off, idx = knn.knn_exact(nd.X, 30)
        W, st = rbffd.weights(nd.X, off, idx, 3, ("lap", "dx", "dy"))
        assert np.all(st == 0)
        s = np.full(nd.N, 5.0)
        us = _steady_system(nd, off, idx, W, kind, normals, g, s)
        errs.append(np.abs(us - hc.annulus_steady(nd.X, neumann_inner=neumann_inner)).max())
        dt = 0.02 * h * h
        u1 = explicit.explicit_step(off, idx, W[0], W[1:], kind, normals, us, dt, g=g, s=s)
        # the step changes u by dt * (residual of the steady equations) only
        assert np.abs(u1 - us).max() < 1e-9 * max(1.0, np.abs(us).max())
    assert errs[1] < errs[0] and errs[1] < (0.15 if neumann_inner else 0.01), errs
