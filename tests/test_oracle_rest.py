"""Pins of the remaining oracle parts: CSR (Sec. 2.3.2), mixed-precision refinement,
surrogate network (bfloat16 rounding, GELU, gradients, Adam), projection, and the
convergence behaviour of the whole method (Sec. 3.2 error study, Sec. 5 Poisson)."""
import math

import numpy as np
import pytest
import torch

import nodesets as ns
from oracle import csr, knn, mlp, poisson, project, rbffd, refine


# ------------------------------------------------------------------------- CSR
def test_csr_matches_stencil_sums():
    nd = ns.disk(0.06, 11)
    sizes = np.random.default_rng(1).integers(6, 20, size=nd.N)
    off, idx = knn.knn_exact(nd.X, sizes)
    W, st = rbffd.weights(nd.X, off, idx, 2, ("lap", "dx"))
    rp, col, vals = csr.to_csr(off, idx, W)
    assert rp[-1] == sizes.sum() and np.array_equal(rp, off)
    for i in range(nd.N):
        c = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0)
        assert sorted(c.tolist()) == sorted(idx[off[i]:off[i + 1]].tolist())
    u = np.random.default_rng(2).normal(size=nd.N)
    row = np.repeat(np.arange(nd.N), sizes)
    for r in range(2):
        direct = np.bincount(row, weights=W[r] * u[idx], minlength=nd.N)
        M = csr.to_scipy(rp, col, vals[r], nd.N)
        np.testing.assert_allclose(M @ u, direct, rtol=1e-12, atol=1e-9)


# ------------------------------------------------------------- refinement (IR)
def test_ir_accepts_well_conditioned_and_matches_lu():
    nd = ns.cube_minus_sphere(1.0 / 12, 4)
    off, idx = knn.knn_exact(nd.X, 35)
    for i in [0, 17, nd.N - 1]:
        Xs = nd.X[idx[off[i]:off[i + 1]]]
        K, B, s = rbffd.assemble(Xs[None], 3, ("lap", "dx", "dy", "dz"))
        x, it, ok = refine.ir_solve(K[0], B[0])
        assert ok and 1 <= it <= 4
        ref = np.linalg.solve(K[0], B[0])
        assert np.abs(x - ref).max() <= 1e-11 * np.abs(ref).max()


def test_ir_forced_fallbacks():
    Xs = ns.disk(0.1, 1).X[:15]
    K, B, s = rbffd.assemble(Xs[None], 2, ("lap",))
    assert refine.ir_solve(K[0], B[0], max_iters=0)[2] is False
    # duplicate node: singular in float64 as well -> never accepted
    Xd = np.vstack([Xs[:14], Xs[3:4]])
    K, B, s = rbffd.assemble(Xd[None], 2, ("lap",))
    assert refine.ir_solve(K[0], B[0])[2] is False


# ------------------------------------------------------------------ bfloat16
def test_bf16_rounding_against_torch():
    rng = np.random.default_rng(5)
    x32 = (rng.normal(size=20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x32.astype(np.float64)), ref)
    # ties to even
    assert mlp.bf16(1.0 + 2.0 ** -8) == 1.0
    assert mlp.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert mlp.bf16(-(1.0 + 3 * 2.0 ** -8)) == -(1.0 + 2.0 ** -6)


def test_gelu_against_torch():
    z = np.linspace(-8, 8, 1001)
    ref = torch.nn.functional.gelu(torch.from_numpy(z)).numpy()
    np.testing.assert_allclose(mlp.gelu(z), ref, rtol=1e-14, atol=1e-15)
    zt = torch.from_numpy(z).requires_grad_(True)
    torch.nn.functional.gelu(zt).sum().backward()
    np.testing.assert_allclose(mlp.gelu_prime(z), zt.grad.numpy(), rtol=1e-12, atol=1e-14)


# --------------------------------------------------------------- MLP gradients
def small_problem(B=16, seed=0):
    p = ns.surrogate_init(seed)
    rng = np.random.default_rng(seed + 1)
    for L in range(1, 5):
        p[f"b{L}"] = rng.normal(scale=0.1, size=p[f"b{L}"].shape)
    x = rng.uniform(-1, 1, size=(B, 30))
    t = rng.normal(size=(B, 15))
    return p, x, t


def test_mlp_gradients_finite_differences():
    p, x, t = small_problem()
    loss, g, _ = mlp.loss_and_grads(p, x, t, rounding=False)
    rng = np.random.default_rng(3)
    for k in ["W1", "b1", "W2", "b3", "W4", "b4"]:
        for _ in range(4):
            ix = tuple(rng.integers(0, s) for s in p[k].shape)
            eps = 1e-6
            pp = {a: b.copy() for a, b in p.items()}
            pp[k][ix] += eps
            lp = mlp.loss_and_grads(pp, x, t, rounding=False)[0]
            pp[k][ix] -= 2 * eps
            lm = mlp.loss_and_grads(pp, x, t, rounding=False)[0]
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - g[k][ix]) <= 1e-6 * max(1e-3, abs(fd)), (k, fd, g[k][ix])


def test_mlp_matches_torch_autograd_without_rounding():
    p, x, t = small_problem(B=32, seed=4)
    loss, g, y = mlp.loss_and_grads(p, x, t, rounding=False)
    tp = {k: torch.from_numpy(v.copy()).requires_grad_(True) for k, v in p.items()}
    h = torch.from_numpy(x)
    for L in range(1, 5):
        h = h @ tp[f"W{L}"].T + tp[f"b{L}"]
        if L < 4:
            h = torch.nn.functional.gelu(h)
    lt = torch.mean((h - torch.from_numpy(t)) ** 2)
    lt.backward()
    assert abs(lt.item() - loss) <= 1e-12 * loss
    for k in p:
        np.testing.assert_allclose(g[k], tp[k].grad.numpy(), rtol=1e-9, atol=1e-14)


def test_rounded_network_close_to_plain():
    p, x, t = small_problem(B=64, seed=6)
    y1, _ = mlp.forward(p, x, rounding=True)
    y0, _ = mlp.forward(p, x, rounding=False)
    assert np.abs(y1 - y0).max() <= 0.05 * np.abs(y0).max()


def test_adam_first_step_closed_form():
    p = {"a": np.array([1.0, -2.0, 3.0])}
    g = {"a": np.array([0.5, -1e-3, 0.0])}
    mlp.adam_step(p, g, {}, lr=1e-2)
    # first step: m_hat = g, v_hat = g^2 -> update = lr * g / (|g| + eps)
    np.testing.assert_allclose(p["a"], [1.0 - 1e-2 * 0.5 / (0.5 + 1e-8),
                                        -2.0 + 1e-2 * 1e-3 / (1e-3 + 1e-8), 3.0], rtol=1e-15)


# ------------------------------------------------------------------ projection
def test_projection_is_min_norm_correction():
    nd = ns.disk(0.0404, 1001)
    off, idx = knn.knn_exact(nd.X, 15)
    F, s = mlp.stencil_features(nd.X, off, idx, np.arange(0, nd.N, 50))
    Xh = F.reshape(F.shape[0], 15, 2)
    y = np.random.default_rng(0).normal(size=(F.shape[0], 15)) * 10
    lq = project.lap_lq(2, 2)
    w, rho = project.project(y, Xh, 2, lq)
    assert rho.max() < 1e-12
    for b in range(0, F.shape[0], 7):
        # independent route: minimum-norm correction by the pseudo-inverse of Q^T
        Q = np.array([[1, a, c, a * a, a * c, c * c] for a, c in Xh[b]])
        ref = y[b] + np.linalg.pinv(Q.T) @ (np.array([0, 0, 0, 2, 0, 2.0]) - Q.T @ y[b])
        np.testing.assert_allclose(w[b], ref, rtol=1e-9, atol=1e-9)
    # the exact weights are a fixed point
    Wt, _ = rbffd.weights(nd.X, off, idx, 2, ("lap",))
    nodes = np.arange(0, nd.N, 50)
    ex = np.stack([Wt[0, off[i]:off[i + 1]] for i in nodes]) * (s[:, None] ** 2)
    w2, _ = project.project(ex, Xh, 2, lq)
    np.testing.assert_allclose(w2, ex, rtol=1e-8, atol=1e-8)


# ------------------------------------------------------------------ convergence
def test_laplacian_error_order_regular_grid():
    """Sec. 3.2 study, setup 5 (PHS r^5, degree 2, 12 closest nodes) and r^3 with 15:
    e_h decays at least like h^(P-1) = h."""
    for k, n in [(5, 12), (3, 15)]:
        errs, hs = [], [1 / 16, 1 / 32, 1 / 64]
        for h in hs:
            g = ns.unit_square_grid(h)
            off, idx = knn.knn_exact(g.X, n)
            W, st = rbffd.weights(g.X, off, idx, 2, ("lap",), phs_power=k)
            errs.append(poisson.lap_error(g.X, off, idx, W[0]))
        order = np.polyfit(np.log(hs), np.log(errs), 1)[0]
        assert order >= 0.9, (k, n, errs)


@pytest.mark.parametrize("d,n,hs,slope_min", [(2, 9, (0.08, 0.04, 0.02), 0.85),
                                              (3, 35, (0.2, 0.14, 0.1), 0.5)])
def test_poisson_convergence_rate(d, n, hs, slope_min):
    """Sec. 5: the solution error decays like N^(-2/d)."""
    Ns, errs = [], []
    for h in hs:
        a = ns.annulus(h, 7, d)
        off, idx = knn.knn_exact(a.X, n)
        W, st = rbffd.weights(a.X, off, idx, 2, ("lap",))
        assert st.max() == 0 and st.min() == 0
        u, err = poisson.solve_dirichlet(a.X, a.is_boundary, off, idx, W[0])
        Ns.append(a.N)
        errs.append(err)
    slope = -np.polyfit(np.log(Ns), np.log(errs), 1)[0]
    assert slope >= slope_min * (2.0 / d), (Ns, errs, slope)


def test_canonical_features_frame_and_invariance():
    """Canonical inputs: node 1 on +x, node 2 in y >= 0, norms kept, and the same features
    for a rotated and reflected copy of the node set (up to rounding)."""
    nd = ns.disk(0.0404, 1001)
    off, idx = knn.knn_exact(nd.X, 15)
    nodes = np.arange(0, nd.N, 13)
    F, s = mlp.stencil_features(nd.X, off, idx, nodes, canonical=True)
    G, s0 = mlp.stencil_features(nd.X, off, idx, nodes, canonical=False)
    F3, G3 = F.reshape(-1, 15, 2), G.reshape(-1, 15, 2)
    assert np.array_equal(s, s0)
    assert np.abs(F3[:, 1, 1]).max() <= 1e-15 and np.all(F3[:, 1, 0] > 0) and np.all(F3[:, 2, 1] >= -1e-15)
    np.testing.assert_allclose(np.linalg.norm(F3, axis=-1), np.linalg.norm(G3, axis=-1), atol=1e-15)
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]]) @ np.diag([1.0, -1.0])
    Fr, _ = mlp.stencil_features(nd.X @ R.T + 0.3, off, idx, nodes, canonical=True)
    np.testing.assert_allclose(Fr, F, atol=1e-13)
    # the Laplacian weights computed from the canonical coordinates are those of the stencil
    Wt, _ = rbffd.weights(nd.X, off, idx, 2, ("lap",))
    for k, i in enumerate(nodes[:20]):
        Xs = F3[k] * s[k]
        w2, _ = rbffd.weights(Xs, np.array([0, 15]), np.arange(15), 2, ("lap",))
        np.testing.assert_allclose(w2[0], Wt[0, off[i]:off[i + 1]], rtol=1e-9, atol=1e-9 * np.abs(w2[0]).max())
