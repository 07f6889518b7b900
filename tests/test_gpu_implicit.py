"""GPU implicit solution (Sec. 2.3.2, Sec. 5) against the oracle.

rbf_assemble_implicit is compared entry by entry with oracle/implicit.py
(interior and Dirichlet rows are copies: bit-equal; Neumann rows sum d
products: the rounding bound 2 d eps sum_l |n_l w_l|).  rbf_bicgstab is
compared with the oracle's direct solve of the oracle's system: the residual
the solver monitors is recomputed on the host, and the solution must agree
with the direct one to the accuracy the residual implies.  The whole GPU path
(stencils, weights, assembly, BiCGStab) repeats the manufactured Poisson
problem of Sec. 5 at the paper's convergence rate.
"""
import math

import numpy as np
import pytest
import torch

import nodesets as ns
from oracle import implicit, knn, poisson, rbffd
import heat_cases as hc

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def _rb():
    import paper_1912_13282_amd as rb
    return rb


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _annulus_problem(h, d=2, n=30, P=3, neumann=True, seed=5):
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
    f = poisson.lap_u0(X)
    return nd, kind, normals, off, idx.astype(np.int32), W, f, g, u0


@pytest.mark.parametrize("d", [2, 3])
def test_assemble_implicit_parity(gpu, d):
    rb = _rb()
    nd, kind, normals, off, idx, W, f, g, _ = _annulus_problem(0.05 if d == 2 else 0.15, d=d,
                                                                n=30 if d == 2 else 35, P=3)
    vo, ro = implicit.assemble(off, idx, W[0], W[1:], kind, normals, f=f, g=g)
    Wt = _t(W, gpu)
    vals, rhs = rb.assemble_implicit(_t(off, gpu), _t(idx, gpu), Wt[0], _t(kind, gpu), w_grad=Wt[1:],
                                     normals=_t(normals, gpu), f=_t(f, gpu), g=_t(g, gpu))
    vg, rg = vals.cpu().numpy(), rhs.cpu().numpy()
    assert np.array_equal(rg, ro)
    row = np.repeat(np.arange(nd.N), np.diff(off))
    ne = kind[row] == hc.NEUMANN
    assert np.array_equal(vg[~ne], vo[~ne])
    bound = 2 * d * EPS * sum(np.abs(normals[row, l] * W[1 + l]) for l in range(d))
    assert np.all(np.abs(vg[ne] - vo[ne]) <= bound[ne])
    # f and g omitted: zero right-hand side
    _, r0 = rb.assemble_implicit(_t(off, gpu), _t(idx, gpu), Wt[0], _t(kind, gpu), w_grad=Wt[1:],
                                 normals=_t(normals, gpu))
    assert torch.count_nonzero(r0).item() == 0


def test_assemble_implicit_invalid_rows(gpu):
    rb = _rb()
    nd, kind, normals, off, idx, W, f, g, _ = _annulus_problem(0.1)
    kind = kind.copy()
    idx2 = idx.copy()
    inter = np.where(kind == hc.INTERIOR)[0]
    dirich = np.where(kind == hc.DIRICHLET)[0]
    neu = np.where(kind == hc.NEUMANN)[0]
    kind[inter[0]] = 9
    idx2[off[dirich[0]]] = idx2[off[dirich[0]] + 1]   # position 0 not the node itself
    idx2[off[neu[0]]] = idx2[off[neu[0]] + 1]
    Wt = _t(W, gpu)
    vals, rhs = rb.assemble_implicit(_t(off, gpu), _t(idx2, gpu), Wt[0], _t(kind, gpu), w_grad=Wt[1:],
                                     normals=_t(normals, gpu), f=_t(f, gpu), g=_t(g, gpu))
    vg, rg = vals.cpu().numpy(), rhs.cpu().numpy()
    bad = [inter[0], dirich[0], neu[0]]
    assert np.all(np.isnan(rg[bad]))
    for i in bad:
        assert np.all(np.isnan(vg[off[i]:off[i + 1]]))
    good = np.setdiff1d(np.arange(nd.N), bad)
    assert not np.any(np.isnan(rg[good]))
    # Neumann rows without gradient weights
    _, r2 = rb.assemble_implicit(_t(off, gpu), _t(idx, gpu), Wt[0], _t(np.where(kind == 9, 0, kind).astype(np.uint8),
                                                                       gpu), f=_t(f, gpu), g=_t(g, gpu))
    assert np.all(np.isnan(r2.cpu().numpy()[neu]))


def _scaled_residual(off, idx, vals, rhs, x, jacobi=True):
    M = implicit.matrix(off, idx, vals)
    dinv = 1.0 / M.diagonal() if jacobi else np.ones(M.shape[0])
    return np.linalg.norm(dinv * (rhs - M @ x)) / np.linalg.norm(dinv * rhs)


# 2D with Neumann rows needs the Jacobi scaling (about 4,200 iterations here);
# the Dirichlet problems converge in a few hundred either way
@pytest.mark.parametrize("d,precond,neumann", [(2, "jacobi", True), (2, "none", False), (3, "jacobi", False),
                                               (3, "none", False), (2, "block_jacobi", True),
                                               (3, "block_jacobi", False)])
def test_bicgstab_parity_with_direct_solve(gpu, d, precond, neumann):
    rb = _rb()
    nd, kind, normals, off, idx, W, f, g, u0 = _annulus_problem(0.025 if d == 2 else 0.12, d=d,
                                                                 n=30 if d == 2 else 35, P=3, neumann=neumann)
    vals, rhs = implicit.assemble(off, idx, W[0], W[1:], kind, normals, f=f, g=g)
    ud = implicit.solve(off, idx, vals, rhs)
    tol = 1e-12
    n_max = int(np.diff(off).max())
    pc = rb.block_jacobi(_t(nd.X, gpu), _t(off, gpu), _t(idx, gpu), _t(vals, gpu)) if precond == "block_jacobi" \
        else None
    x, info = rb.bicgstab(_t(off, gpu), _t(idx, gpu), _t(vals, gpu), n_max, _t(rhs, gpu), tol=tol, max_iter=20000,
                          precond=precond, pc=pc)
    assert info["status"] == rb.SOLVE_CONVERGED, info
    xh = x.cpu().numpy()
    # the monitored residual is updated by the recursion, which drifts from
    # b - M x over the thousand-odd iterations of the Neumann problem; a converged
    # x is checked against its recomputed residual (in the monitored norm) and
    # restarted from when that is above 2 tol, so the recomputed residual here
    # is within 2 tol up to the rounding of forming it
    res = _scaled_residual(off, idx, vals, rhs, xh, jacobi=precond == "jacobi")
    assert res <= 2.5 * tol, (res, info)
    assert info["residual"] <= tol
    M = implicit.matrix(off, idx, vals)
    # the unscaled residual recomputed on the host, to the rounding of forming r - M x
    # (n-term sums of |M||x| plus |r|, in another order on each side)
    n_row = int(np.diff(off).max())
    slack = 2 * (n_row + 2) * EPS * np.linalg.norm(abs(M) @ np.abs(xh) + np.abs(rhs)) / np.linalg.norm(rhs)
    assert abs(info["true_residual"] - np.linalg.norm(rhs - M @ xh) / np.linalg.norm(rhs)) <= slack
    # the direct solution, to the accuracy that residual allows (condition number below 1e5 here)
    assert np.abs(xh - ud).max() <= 1e5 * 10 * tol * np.abs(ud).max(), np.abs(xh - ud).max()
    assert np.abs(xh - u0).max() < 0.05
    # deterministic: a second solve (and a second preconditioner set-up) is bit-identical
    if pc is not None:
        pc = rb.block_jacobi(_t(nd.X, gpu), _t(off, gpu), _t(idx, gpu), _t(vals, gpu))
    x2, info2 = rb.bicgstab(_t(off, gpu), _t(idx, gpu), _t(vals, gpu), n_max, _t(rhs, gpu), tol=tol, max_iter=20000,
                            precond=precond, pc=pc)
    assert torch.equal(x, x2) and info2["iterations"] == info["iterations"]
    print(f"  {d}D {precond} neumann={neumann}: {info['iterations']} iterations", flush=True)


@pytest.mark.parametrize("d,h,n", [(2, 0.01, 9), (3, 0.05, 35)])
def test_block_jacobi_cuts_iterations(gpu, d, h, n):
    """The Sec. 5 Dirichlet problem (degree 2): block-Jacobi BiCGStab converges to the
    same solution as Jacobi in fewer iterations (2D: under 55% of Jacobi's; 3D, where
    the 35-node stencils reach further out of a 64-node block: under 75%)."""
    rb = _rb()
    nd = ns.annulus(h, 1006, d=d)
    off, idx = knn.knn_exact(nd.X, n)
    W, _ = rbffd.weights(nd.X, off, idx, 2, ("lap",))
    kind = np.where(nd.is_boundary, hc.DIRICHLET, hc.INTERIOR).astype(np.uint8)
    vals, rhs = implicit.assemble(off, idx.astype(np.int32), W[0], None, kind, None, f=poisson.lap_u0(nd.X),
                                  g=poisson.u0(nd.X))
    T = [_t(a, gpu) for a in (off, idx.astype(np.int32), vals, rhs)]
    xj, ij = rb.bicgstab(*T[:3], n, T[3], tol=1e-10, max_iter=20000, precond="jacobi")
    pc = rb.block_jacobi(_t(nd.X, gpu), *T[:3])
    xb, ib = rb.bicgstab(*T[:3], n, T[3], tol=1e-10, max_iter=20000, precond="block_jacobi", pc=pc)
    print(f"  {d}D N={nd.N}: Jacobi {ij['iterations']} iterations, block-Jacobi {ib['iterations']}", flush=True)
    assert ij["status"] == rb.SOLVE_CONVERGED and ib["status"] == rb.SOLVE_CONVERGED
    assert ib["iterations"] <= (0.55 if d == 2 else 0.75) * ij["iterations"]
    u0 = poisson.u0(nd.X)
    ej, eb = np.abs(xj.cpu().numpy() - u0).max(), np.abs(xb.cpu().numpy() - u0).max()
    assert abs(eb - ej) <= 1e-3 * ej


def test_block_jacobi_order_is_deterministic_with_a_crowded_cell(gpu):
    """The node order of the block-Jacobi preconditioner is ascending ids inside
    every cell, also in a cell far above the average fill (400 coincident-ish
    nodes): two set-ups give the same bytes, the order is a permutation, and the
    crowded cell's ids come out sorted."""
    rb = _rb()
    rng = np.random.default_rng(11)
    X = np.concatenate([rng.random((3000, 2)), 0.5 + 1e-9 * rng.random((400, 2))])
    perm_in = rng.permutation(X.shape[0])
    X = np.ascontiguousarray(X[perm_in])
    N = X.shape[0]
    off = np.arange(N + 1, dtype=np.int64)
    idx = np.arange(N, dtype=np.int32)
    vals = np.full(N, 2.0)
    T = [_t(a, gpu) for a in (X, off, idx, vals)]
    pc1 = rb.block_jacobi(*T)
    pc2 = rb.block_jacobi(*T)
    # the order, its inverse, the float16 inverses and their scales (regions
    # aligned to 256 bytes; the padding between them and the set-up's scratch
    # at the end are not part of the result)
    al = lambda b: (b + 255) // 256 * 256  # noqa: E731
    nb = (N + 63) // 64
    o = 0
    for size in (4 * N, 4 * N, 2 * 64 * 64 * nb, 4 * 64 * nb):
        assert torch.equal(pc1[o:o + size], pc2[o:o + size])
        o += al(size)
    order = pc1[: 4 * N].cpu().numpy().view(np.int32)
    assert np.array_equal(np.sort(order), np.arange(N))
    crowd = np.nonzero(perm_in >= 3000)[0]              # ids of the clustered nodes
    pos = np.nonzero(np.isin(order, crowd))[0]
    assert pos.max() - pos.min() + 1 >= 400
    seg = order[pos.min():pos.max() + 1]
    assert np.all(np.diff(seg) > 0)
    # and the preconditioner solves the diagonal system exactly
    x, info = rb.bicgstab(*T[1:], 1, _t(np.ones(N), gpu), tol=1e-12, precond="block_jacobi", pc=pc1)
    assert info["status"] == rb.SOLVE_CONVERGED and np.allclose(x.cpu().numpy(), 0.5)


def test_3d_neumann_reports_failure(gpu):
    """Closest-node Neumann rows in 3D: a few percent have a normal-derivative weight
    at the node of the wrong sign, the operator is unstable and no preconditioner
    makes BiCGStab converge; the solver must say so (never report CONVERGED)."""
    rb = _rb()
    nd, kind, normals, off, idx, W, f, g, u0 = _annulus_problem(0.08, d=3, n=35, P=2, neumann=True)
    vals, rhs = implicit.assemble(off, idx, W[0], W[1:], kind, normals, f=f, g=g)
    T = [_t(a, gpu) for a in (off, idx, vals, rhs)]
    for precond in ("jacobi", "block_jacobi"):
        pc = rb.block_jacobi(_t(nd.X, gpu), *T[:3]) if precond == "block_jacobi" else None
        x, info = rb.bicgstab(*T[:3], 35, T[3], tol=1e-10, max_iter=3000, precond=precond, pc=pc)
        print(f"  {precond}: {info}", flush=True)
        assert info["status"] in (rb.SOLVE_MAXITER, rb.SOLVE_DIVERGED, rb.SOLVE_BREAKDOWN)


@pytest.mark.parametrize("precond", ["jacobi", "block_jacobi"])
def test_bicgstab_csr_with_ragged_rows(gpu, precond):
    """The solver on CSR input: columns ascending (the diagonal anywhere in a row),
    explicit zeros dropped so that Dirichlet rows hold one entry (block-Jacobi:
    the copy in block order has rows of every length)."""
    rb = _rb()
    nd, kind, normals, off, idx, W, f, g, u0 = _annulus_problem(0.025, neumann=False)
    vals, rhs = implicit.assemble(off, idx, W[0], W[1:], kind, normals, f=f, g=g)
    M = implicit.matrix(off, idx, vals)
    M.eliminate_zeros()
    M.sort_indices()
    lens = np.diff(M.indptr)
    assert lens.min() == 1 and lens.max() == 30
    ud = implicit.solve(off, idx, vals, rhs)
    tol = 1e-12
    T = [_t(M.indptr.astype(np.int64), gpu), _t(M.indices.astype(np.int32), gpu), _t(M.data, gpu)]
    pc = rb.block_jacobi(_t(nd.X, gpu), *T) if precond == "block_jacobi" else None
    x, info = rb.bicgstab(*T, 30, _t(rhs, gpu), tol=tol, max_iter=20000, precond=precond, pc=pc)
    assert info["status"] == rb.SOLVE_CONVERGED, info
    xh = x.cpu().numpy()
    dinv = 1.0 / M.diagonal() if precond == "jacobi" else np.ones(nd.N)
    assert np.linalg.norm(dinv * (rhs - M @ xh)) / np.linalg.norm(dinv * rhs) <= 10 * tol
    assert np.abs(xh - ud).max() <= 1e5 * 10 * tol * np.abs(ud).max()



@pytest.mark.parametrize("precond", ["jacobi", "block_jacobi"])
def test_bicgstab_restarts_from_a_drifted_residual(gpu, precond):
    """A start 1e8 times too large: the recursively updated residual drifts from
    b - M x by the rounding of the first, huge residuals (about 1e-8 of |b|), far above
    the 1e-12 tolerance.  The check of the converged x must restart from it and end
    with the recomputed residual within 2 tol."""
    rb = _rb()
    nd, kind, normals, off, idx, W, f, g, u0 = _annulus_problem(0.12, d=3, n=35, P=3, neumann=False)
    vals, rhs = implicit.assemble(off, idx, W[0], W[1:], kind, normals, f=f, g=g)
    ud = implicit.solve(off, idx, vals, rhs)
    tol = 1e-12
    n_max = int(np.diff(off).max())
    x0 = 1e8 * np.random.default_rng(3).standard_normal(nd.N)
    pc = rb.block_jacobi(_t(nd.X, gpu), _t(off, gpu), _t(idx, gpu), _t(vals, gpu)) if precond == "block_jacobi" \
        else None
    x, info = rb.bicgstab(_t(off, gpu), _t(idx, gpu), _t(vals, gpu), n_max, _t(rhs, gpu), x=_t(x0, gpu), tol=tol,
                          max_iter=20000, precond=precond, pc=pc)
    assert info["status"] == rb.SOLVE_CONVERGED, info
    xh = x.cpu().numpy()
    res = _scaled_residual(off, idx, vals, rhs, xh, jacobi=precond == "jacobi")
    assert res <= 2.5 * tol, (res, info)
    assert np.abs(xh - ud).max() <= 1e5 * 10 * tol * np.abs(ud).max(), np.abs(xh - ud).max()


@pytest.mark.parametrize("precond", ["jacobi", "block_jacobi"])
def test_bicgstab_outcomes(gpu, precond):
    rb = _rb()
    nd, kind, normals, off, idx, W, f, g, _ = _annulus_problem(0.05)
    vals, rhs = implicit.assemble(off, idx, W[0], W[1:], kind, normals, f=f, g=g)
    n_max = int(np.diff(off).max())
    to = lambda a: _t(a, gpu)  # noqa: E731
    pc = rb.block_jacobi(to(nd.X), to(off), to(idx), to(vals)) if precond == "block_jacobi" else None
    kw = dict(precond=precond, pc=pc)
    # iteration limit
    x, info = rb.bicgstab(to(off), to(idx), to(vals), n_max, to(rhs), tol=1e-14, max_iter=3, **kw)
    assert info["status"] == rb.SOLVE_MAXITER and info["iterations"] == 3
    # the exact solution as the initial guess: converged without iterating, x
    # returned bit for bit (block-Jacobi: through the copy in block order and back)
    ud = implicit.solve(off, idx, vals, rhs)
    x, info = rb.bicgstab(to(off), to(idx), to(vals), n_max, to(rhs), x=to(ud), tol=1e-6, **kw)
    assert info["status"] == rb.SOLVE_CONVERGED and info["iterations"] == 0
    assert np.array_equal(x.cpu().numpy(), ud)
    # zero right-hand side from zero: converged at once, x stays zero
    x, info = rb.bicgstab(to(off), to(idx), to(vals), n_max, torch.zeros(nd.N, dtype=torch.float64, device=gpu),
                          **kw)
    assert info["status"] == rb.SOLVE_CONVERGED and info["iterations"] == 0 and torch.count_nonzero(x).item() == 0
    if precond == "jacobi":
        # a zero diagonal entry with Jacobi scaling
        v2 = vals.copy()
        i = np.where(kind == hc.INTERIOR)[0][3]
        v2[off[i]] = 0.0
        x, info = rb.bicgstab(to(off), to(idx), to(v2), n_max, to(rhs), **kw)
        assert info["status"] == rb.SOLVE_BADDIAG
    # non-finite input: breakdown, never a hang
    r2 = rhs.copy()
    r2[5] = np.nan
    x, info = rb.bicgstab(to(off), to(idx), to(vals), n_max, to(r2), **kw)
    assert info["status"] == rb.SOLVE_BREAKDOWN
    # a row with an invalid range (end before start) or an index outside [0, N)
    # gives a NaN row product: breakdown
    # (Jacobi: the row has no diagonal entry either)
    o2 = off.copy()
    o2[7] = o2[8] + 1
    x, info = rb.bicgstab(to(o2), to(idx), to(vals), n_max, to(rhs), **kw)
    assert info["status"] == (rb.SOLVE_BADDIAG if precond == "jacobi" else rb.SOLVE_BREAKDOWN)
    i2 = idx.copy()
    i2[off[11] + 2] = nd.N + 5
    x, info = rb.bicgstab(to(off), to(i2), to(vals), n_max, to(rhs), **kw)
    assert info["status"] == rb.SOLVE_BREAKDOWN
    with pytest.raises(rb.RbfError):
        rb.bicgstab(to(off), to(idx), to(vals), n_max, to(rhs), precond="ilu")


def test_gpu_poisson_at_the_papers_rate(gpu):
    """Sec. 5 on the GPU: annulus, u_0 = prod sin(pi x_a), n = 9 in 2D with degree 2;
    stencils, weights, assembly and BiCGStab on the device; error ~ N^(-1)."""
    rb = _rb()
    Ns, errs = [], []
    for h in (0.02, 0.01, 0.005):
        nd = ns.annulus(h, 5, d=2)
        N, n = nd.N, 9
        X = _t(nd.X, gpu)
        off = _t(ns.offsets_from_sizes(np.full(N, n, dtype=np.int64)), gpu)
        idx = rb.select_stencils(X, off, n)
        w, st = rb.compute_weights(X, off, idx, n, 2, ("lap",))
        assert int((st != 0).sum()) == 0
        kind = _t(np.where(nd.is_boundary, hc.DIRICHLET, hc.INTERIOR).astype(np.uint8), gpu)
        u0 = poisson.u0(nd.X)
        vals, rhs = rb.assemble_implicit(off, idx, w[0], kind, f=_t(poisson.lap_u0(nd.X), gpu), g=_t(u0, gpu))
        x, info = rb.bicgstab(off, idx, vals, n, rhs, tol=1e-11, max_iter=50000)
        assert info["status"] == rb.SOLVE_CONVERGED, info
        Ns.append(N)
        errs.append(float(np.abs(x.cpu().numpy() - u0).max()))
    slope = np.polyfit(np.log(Ns), np.log(errs), 1)[0]
    assert -1.4 < slope < -0.7, (Ns, errs, slope)
