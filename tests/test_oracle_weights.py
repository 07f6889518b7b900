"""Pins of the oracle RBF-FD weights, eq. (rbf-system-aug), against what the
mathematics fixes independently of the oracle's own formulas:

* unisolvent n = m stencils: textbook finite-difference stars (closed form);
* polynomial reproduction checked with finite differences of random polynomials;
* w^T u equals the operator applied to the augmented interpolant of u, where the
  interpolant is built and differentiated here (finite differences), not by the oracle;
* translation / rotation / dilation / permutation covariance, D4 symmetry;
* singular systems flagged.
"""
import math

import numpy as np
import pytest

import nodesets as ns
from oracle import knn, rbffd

RNG = np.random.default_rng(12345)


def jittered_stencil(d, n, rng, h=0.01):
    """A centre plus n-1 nearest nodes of a jittered lattice patch around it."""
    k = 4
    g = np.stack(np.meshgrid(*(np.arange(-k, k + 1),) * d, indexing="ij"), -1).reshape(-1, d) * h
    g = g + rng.uniform(-0.25 * h, 0.25 * h, size=g.shape)
    c = g[len(g) // 2]
    o = np.argsort(np.sum((g - c) ** 2, axis=1))
    return g[o[:n]] + rng.uniform(-3, 3, size=d)          # arbitrary translation


# ---------------------------------------------------------------- closed forms
def golden_stars():
    """Closed-form star weights from tests/golden/fd_stars.txt."""
    import os
    out = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "fd_stars.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split(":", 1)
                if k.endswith("offsets"):
                    out[k] = np.array([[float(t) for t in p.split()] for p in v.split("|")])
                else:
                    out[k] = np.array([float(t) for t in v.split()])
    return out


@pytest.mark.parametrize("h", [1.0, 0.013, 3.7e-4])
def test_unisolvent_2d_star(h):
    g = golden_stars()
    c = np.array([0.31, -1.7])
    Xs = c + h * g["2d.offsets"]
    W = rbffd.stencil_weights(Xs, 2, ("lap", "dx", "dy"))
    np.testing.assert_allclose(W[0] * h * h, g["2d.lap_h2"], atol=1e-11)
    np.testing.assert_allclose(W[1] * h, g["2d.dx_h"], atol=1e-11)
    np.testing.assert_allclose(W[2] * h, g["2d.dy_h"], atol=1e-11)


@pytest.mark.parametrize("phs", [3, 5])
def test_unisolvent_3d_star(phs):
    g = golden_stars()
    h = 0.02
    Xs = h * g["3d.offsets"]
    W = rbffd.stencil_weights(Xs, 2, ("lap", "dz"), phs_power=phs)
    np.testing.assert_allclose(W[0] * h * h, g["3d.lap_h2"], atol=1e-10)
    np.testing.assert_allclose(W[1] * h, g["3d.dz_h"], atol=1e-10)


def test_monomial_count_and_order():
    for d in (2, 3):
        for P in range(5):
            E = rbffd.monomial_exponents(d, P)
            assert E.shape[0] == math.comb(P + d, d)
            assert len({tuple(e) for e in E}) == E.shape[0]
            assert np.all(np.diff(E.sum(axis=1)) >= 0)
    assert rbffd.monomial_exponents(2, 2).tolist() == [[0, 0], [1, 0], [0, 1], [2, 0], [1, 1], [0, 2]]


# --------------------------------------------------------- finite differences
def fd_op(f, op, d, delta):
    """Operator at 0 by finite differences: 5-point second differences (exact for
    polynomials of degree <= 5), 4-point first differences (exact for degree <= 4)."""
    E = np.eye(d)
    if op == "lap":
        tot = 0.0
        for a in range(d):
            e = E[a] * delta
            tot += (-f(2 * e) + 16 * f(e) - 30 * f(0 * e) + 16 * f(-e) - f(-2 * e)) / (12 * delta ** 2)
        return tot
    a = {"dx": 0, "dy": 1, "dz": 2}[op]
    e = E[a] * delta
    return (-f(2 * e) + 8 * f(e) - 8 * f(-e) + f(-2 * e)) / (12 * delta)


def random_poly(d, P, rng):
    """A random polynomial of total degree <= P in d variables (dense coefficient tensor)."""
    C = rng.normal(size=(P + 1,) * d)
    tot = np.indices(C.shape).sum(axis=0)
    C[tot > P] = 0.0

    def p(x):
        x = np.atleast_2d(x)
        val = np.zeros(x.shape[0])
        for ex in zip(*np.nonzero(C)):
            val += C[ex] * np.prod([x[:, a] ** ex[a] for a in range(d)], axis=0)
        return val
    return p


@pytest.mark.parametrize("d,P,n", [(2, 2, 15), (2, 3, 20), (2, 4, 30), (3, 2, 20), (3, 3, 35), (3, 4, 60)])
def test_polynomial_reproduction(d, P, n):
    rng = np.random.default_rng(100 * d + P)
    Xs = jittered_stencil(d, n, rng)
    ops = ("lap", "dx", "dy") + (("dz",) if d == 3 else ())
    W = rbffd.stencil_weights(Xs, P, ops)
    h = 0.01
    for _ in range(3):
        p = random_poly(d, P, rng)
        vals = p(Xs - Xs[0])
        for c, op in enumerate(ops):
            ref = fd_op(lambda x: p(x)[0], op, d, h)
            got = W[c] @ vals
            scale = np.abs(W[c] * vals).sum() + abs(ref)
            assert abs(got - ref) <= 1e-9 * scale, (op, got, ref)
    # consequences: Laplacian weights sum to 0 and sum w ||o||^2 = 2d
    o2 = np.sum((Xs - Xs[0]) ** 2, axis=1)
    assert abs(W[0].sum()) <= 1e-9 * np.abs(W[0]).sum()
    assert abs(W[0] @ o2 - 2 * d) <= 1e-9 * np.abs(W[0] * o2).sum()


def interpolant(Xh, u, P, k):
    """Augmented PHS interpolant of data u at scaled nodes Xh, built here from the
    definition phi(r) = r^k: s(x) = sum_j c_j ||x - x_j||^k + sum_l d_l x^alpha_l with
    s(x_j) = u_j and sum_j c_j q(x_j) = 0 for every monomial q of degree <= P."""
    n, d = Xh.shape
    exps = [e for e in np.ndindex(*(P + 1,) * d) if sum(e) <= P]
    Qm = np.array([[np.prod([x[a] ** e[a] for a in range(d)]) for e in exps] for x in Xh])
    Am = np.array([[np.linalg.norm(xi - xj) ** k for xj in Xh] for xi in Xh])
    m = len(exps)
    Km = np.block([[Am, Qm], [Qm.T, np.zeros((m, m))]])
    cd = np.linalg.lstsq(Km, np.concatenate([u, np.zeros(m)]), rcond=None)[0]
    c, dd = cd[:n], cd[n:]

    def s(x):
        x = np.asarray(x, float)
        return (c @ (np.linalg.norm(Xh - x, axis=1) ** k)
                + dd @ np.array([np.prod([x[a] ** e[a] for a in range(d)]) for e in exps]))
    return s


@pytest.mark.parametrize("d,P,n,k", [(2, 2, 15, 3), (2, 3, 21, 3), (3, 2, 25, 3), (3, 3, 35, 3), (2, 2, 12, 5)])
def test_weights_apply_operator_to_interpolant(d, P, n, k):
    rng = np.random.default_rng(7 * n + d)
    Xs = jittered_stencil(d, n, rng)
    ops = ("lap", "dx", "dy") + (("dz",) if d == 3 else ())
    W = rbffd.stencil_weights(Xs, P, ops, phs_power=k)
    O = Xs - Xs[0]
    s_ = np.sqrt(np.sum(O * O, axis=1)).max()
    Xh = O / s_
    for _ in range(2):
        u = rng.normal(size=n)
        s = interpolant(Xh, u, P, k)
        for c, op in enumerate(ops):
            order = 2 if op == "lap" else 1
            # Richardson on the step removes the O(delta) term of ||x||^k at its centre
            f1 = fd_op(s, op, d, 2e-3)
            f2 = fd_op(s, op, d, 1e-3)
            ref = (2 * f2 - f1) / s_ ** order
            got = W[c] @ u
            assert abs(got - ref) <= 2e-6 * (np.abs(W[c] * u).sum()), (op, got, ref)


# ------------------------------------------------------------------ covariance
def test_covariance():
    rng = np.random.default_rng(99)
    for d, P, n in [(2, 2, 15), (3, 3, 35)]:
        Xs = jittered_stencil(d, n, rng)
        ops = ("lap", "dx", "dy") + (("dz",) if d == 3 else ())
        W = rbffd.stencil_weights(Xs, P, ops)
        h = 0.01
        tolL = 1e-11 * np.abs(W[0]).max() * h * h
        tolG = 1e-11 * np.abs(W[1:]).max() * h
        # translation
        Wt = rbffd.stencil_weights(Xs + rng.uniform(-10, 10, d), P, ops)
        assert np.abs(Wt[0] - W[0]).max() * h * h <= 1e4 * tolL
        # rotation: lap invariant, gradient rotates (w'_{., j} = R w_{., j})
        Rm, _ = np.linalg.qr(rng.normal(size=(d, d)))
        Wr = rbffd.stencil_weights((Xs - Xs[0]) @ Rm.T, P, ops)
        assert np.abs(Wr[0] - W[0]).max() * h * h <= 10 * tolL
        assert np.abs(Wr[1:] - Rm @ W[1:]).max() * h <= 10 * tolG
        # dilation by c: lap * c^-2, gradient * c^-1
        cf = 3.25
        Wd = rbffd.stencil_weights(Xs * cf, P, ops)
        assert np.abs(Wd[0] * cf * cf - W[0]).max() * h * h <= 10 * tolL
        assert np.abs(Wd[1:] * cf - W[1:]).max() * h <= 10 * tolG
        # permutation of the non-centre nodes permutes the weights
        perm = np.concatenate([[0], 1 + rng.permutation(n - 1)])
        Wp = rbffd.stencil_weights(Xs[perm], P, ops)
        assert np.abs(Wp[:, :] - W[:, perm]).max() <= 1e-10 * np.abs(W).max()


def test_d4_symmetry_3x3():
    h = 0.05
    Xs = h * np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]], float)
    W = rbffd.stencil_weights(Xs, 2, ("lap",))[0] * h * h
    assert np.ptp(W[1:5]) < 1e-12 and np.ptp(W[5:9]) < 1e-12
    assert abs(W.sum()) < 1e-12


def test_singular_system_flagged():
    X = np.array([[0.0, 0.0], [0.1, 0.0], [0.0, 0.1], [0.1, 0.1], [0.2, 0.0], [0.0, 0.2]])
    X = np.vstack([X, X[1]])                   # duplicate node -> two equal rows of K
    off = np.array([0, 7])
    idx = np.array([0, 1, 2, 3, 4, 5, 6])
    W, st = rbffd.weights(X, off, idx, 2, ("lap",))
    assert st[0] == -1 and np.all(np.isnan(W))


def test_batched_equals_single():
    nd = ns.disk(0.1, 3)
    off, idx = knn.knn_exact(nd.X, 15)
    W, st = rbffd.weights(nd.X, off, idx, 2, ("lap", "dx", "dy"))
    assert st.max() == 0
    for i in [0, 5, nd.N - 1]:
        Wi = rbffd.stencil_weights(nd.X[idx[off[i]:off[i + 1]]], 2, ("lap", "dx", "dy"))
        np.testing.assert_array_equal(Wi, W[:, off[i]:off[i + 1]])
