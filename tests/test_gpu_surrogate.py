"""GPU tests of the learned surrogate: MFMA forward and gradients against the
float64 oracle with the same bfloat16 rounding points, Adam, the projection onto
the reproduction conditions, the acceptance thresholds, training with
checkpoint/resume, and the gain of the trained network over the zero-network
ablation (the projection alone)."""
import numpy as np
import pytest
import torch

import nodesets as ns
import paper_1912_13282_amd as rb
from paper_1912_13282_amd import surrogate as S
from oracle import mlp as omlp
from oracle import poisson as opoi
from oracle import project as oproj
from oracle import rbffd as orbf

pytestmark = pytest.mark.gpu


def f32_params(seed, bias_scale=0.1):
    p = ns.surrogate_init(seed)
    rng = np.random.default_rng(seed + 1)
    for L in range(1, 5):
        p[f"b{L}"] = rng.uniform(-bias_scale, bias_scale, size=p[f"b{L}"].shape)
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def rel_stats(got, ref):
    """|got - ref| relative to the largest |ref| of the tensor: (median, max)."""
    e = np.abs(np.asarray(got, np.float64) - ref) / max(float(np.abs(ref).max()), 1e-30)
    return float(np.median(e)), float(e.max())


def disk_features(seed, h=None):
    nd = ns.disk(h or ns.DISK_H, seed)
    off = ns.offsets_from_sizes(np.full(nd.N, 15, np.int64))
    return nd, off


def test_forward_parity(gpu):
    p = f32_params(11)
    nd, off = disk_features(4_000_123)
    from oracle import knn as oknn
    _, idx = oknn.knn_exact(nd.X, 15)
    x, _ = omlp.stencil_features(nd.X, off, idx)
    x = x[:1000].astype(np.float32).astype(np.float64)        # 1000 samples: ragged last tile
    flat = rb.mlp_flatten({k: torch.from_numpy(v) for k, v in p.items()}).to(gpu)
    packed = rb.mlp_pack(flat)
    y = rb.mlp_forward(flat, packed, torch.from_numpy(x).float().to(gpu)).cpu().numpy()
    yo, _ = omlp.forward(p, x, rounding=True)
    med, mx = rel_stats(y, yo)
    print(f"  forward: median rel {med:.2e}, max rel {mx:.2e}", flush=True)
    assert med <= 1e-4 and mx <= 1e-2


def test_gradient_parity(gpu):
    p = f32_params(12)
    rng = np.random.default_rng(5)
    Nrows = 700
    x = rng.uniform(-1, 1, size=(Nrows, 30)).astype(np.float32).astype(np.float64)
    t = rng.normal(size=(Nrows, 15)).astype(np.float32).astype(np.float64)
    sel = rng.permutation(Nrows)[:333]                          # gathered rows, ragged block
    flat = rb.mlp_flatten({k: torch.from_numpy(v) for k, v in p.items()}).to(gpu)
    packed = rb.mlp_pack(flat)
    grads, loss = rb.mlp_grad(flat, packed, torch.from_numpy(x).float().to(gpu), torch.from_numpy(t).float().to(gpu),
                              sel=torch.from_numpy(sel).to(gpu))
    g = rb.mlp_unflatten(grads.cpu())
    lo, go, _ = omlp.loss_and_grads(p, x[sel], t[sel], rounding=True)
    assert abs(float(loss.cpu()) - lo) <= 1e-5 * abs(lo)
    for k in go:
        med, mx = rel_stats(g[k].numpy(), go[k])
        print(f"  d{k}: median rel {med:.2e}, max rel {mx:.2e}", flush=True)
        assert med <= 1e-4 and mx <= 1e-2, k
    # deterministic: the same call gives the same bits
    grads2, _ = rb.mlp_grad(flat, packed, torch.from_numpy(x).float().to(gpu), torch.from_numpy(t).float().to(gpu),
                            sel=torch.from_numpy(sel).to(gpu))
    assert torch.equal(grads, grads2)


def test_adam_parity(gpu):
    p = f32_params(13)
    rng = np.random.default_rng(6)
    flat = rb.mlp_flatten({k: torch.from_numpy(v) for k, v in p.items()}).to(gpu)
    m = torch.zeros_like(flat)
    v = torch.zeros_like(flat)
    po = {k: v_.copy() for k, v_ in p.items()}
    state = {}
    for step in range(1, 4):
        gd = {k: rng.normal(scale=1e-2, size=v_.shape).astype(np.float32).astype(np.float64) for k, v_ in p.items()}
        gflat = rb.mlp_flatten({k: torch.from_numpy(v_) for k, v_ in gd.items()}).to(gpu)
        rb.mlp_adam(flat, gflat, m, v, step, 1e-3)
        po = omlp.adam_step(po, gd, state, 1e-3)
    got = rb.mlp_unflatten(flat.cpu())
    for k in po:
        err = np.abs(got[k].numpy() - po[k]).max()
        assert err <= 1e-6, (k, err)


def _plain_and_stencils(dev, seed=1001):
    nd, off = disk_features(seed)
    X = torch.from_numpy(nd.X).to(dev)
    od = torch.from_numpy(off).to(dev)
    idx = rb.select_stencils(X, od, 15)
    return nd, off, X, od, idx


def test_projection_parity_and_reproduction(gpu):
    """Accept-all threshold: GPU weights = oracle projection of the GPU network output."""
    p = f32_params(14)
    nd, off, X, od, idx = _plain_and_stencils(gpu)
    flat = rb.mlp_flatten({k: torch.from_numpy(v) for k, v in p.items()}).to(gpu)
    rb.surrogate_load(flat)
    w, st = rb.surrogate_weights(X, od, idx, 15, surrogate_tol=1e300, surrogate_corr_tol=1e300)
    feat, _, scale = rb.surrogate_dataset(X, od, idx)
    y = rb.mlp_forward(flat, rb.mlp_pack(flat), feat)
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    assert np.all(st == rb.ST_SURROGATE)
    idx_n = idx.cpu().numpy()
    Xh = (nd.X[idx_n.reshape(-1, 15)] - nd.X[idx_n.reshape(-1, 15)[:, :1]])
    s = np.sqrt((Xh ** 2).sum(-1)).max(1)
    assert np.array_equal(s, scale.cpu().numpy())
    # the features are the oracle's canonical-frame inputs, rounded to float32
    Fo, _ = omlp.stencil_features(nd.X, off, idx_n, canonical=True)
    Fg = feat.cpu().numpy()
    assert np.abs(Fg - Fo.astype(np.float32)).max() <= 2.0 ** -24, np.abs(Fg - Fo.astype(np.float32)).max()
    print(f"  features equal to the oracle's in float32: {np.mean(Fg == Fo.astype(np.float32)):.6f}", flush=True)
    Xh = Xh / s[:, None, None]
    wo, rho = oproj.project(y.cpu().numpy().astype(np.float64), Xh, 2, oproj.lap_lq(2, 2))
    wo = (wo / (s * s)[:, None]).reshape(-1)
    h2 = nd.h[0] ** 2
    E = np.abs(w.cpu().numpy() - wo).max() * h2 / max(1.0, np.abs(wo).max() * h2)
    print(f"  projection E = {E:.2e}, oracle rho max {rho.max():.1e}", flush=True)
    assert E <= 1e-10
    # every accepted stencil reproduces the quadratics (second block row of the system)
    wg = w.cpu().numpy().reshape(-1, 15) * (s * s)[:, None]
    Q = oproj.q_matrix(Xh, 2)
    res = np.abs(np.einsum("bnm,bn->bm", Q, wg) - oproj.lap_lq(2, 2)[None, :]).max() / 2.0
    assert res <= 1e-6


def test_thresholds_and_fallback(gpu):
    p = f32_params(15)
    nd, off, X, od, idx = _plain_and_stencils(gpu)
    flat = rb.mlp_flatten({k: torch.from_numpy(v) for k, v in p.items()}).to(gpu)
    rb.surrogate_load(flat)
    wp, _ = rb.compute_weights(X, od, idx, 15, 2, ("lap",), precision="f64")
    # tolerance 0: a stencil passes only with an exactly zero residual; the rest are solved plainly
    w0, s0 = rb.surrogate_weights(X, od, idx, 15, surrogate_tol=0.0, surrogate_corr_tol=1e300)
    s0 = s0.cpu().numpy()
    rej = s0 == rb.ST_SURROGATE_REJECTED
    assert np.all((s0 == rb.ST_SURROGATE) | rej) and rej.mean() >= 0.99
    wr = w0.cpu().numpy().reshape(-1, 15)[rej]
    assert np.array_equal(wr, wp[0].cpu().numpy().reshape(-1, 15)[rej])   # the plain kernel, bit for bit
    # tolerance infinity: nothing rejected
    _, s1 = rb.surrogate_weights(X, od, idx, 15, surrogate_tol=1e300, surrogate_corr_tol=1e300)
    assert np.all(s1.cpu().numpy() == rb.ST_SURROGATE)
    # stencils that are not 15-node go to the plain solve (sizes 15 and 16 mixed)
    sizes = np.where(np.arange(nd.N) % 7 == 0, 16, 15)
    off2 = ns.offsets_from_sizes(sizes)
    od2 = torch.from_numpy(off2).to(gpu)
    idx2 = rb.select_stencils(X, od2, 16)
    w2, s2 = rb.surrogate_weights(X, od2, idx2, 16, surrogate_tol=1e300, surrogate_corr_tol=1e300)
    s2 = s2.cpu().numpy()
    assert np.all(s2[sizes == 16] == rb.ST_SURROGATE_REJECTED) and np.all(s2[sizes == 15] == rb.ST_SURROGATE)
    wo, _ = orbf.weights(nd.X, off2, idx2.cpu().numpy(), 2, ("lap",))
    pos = np.concatenate([np.arange(off2[i], off2[i + 1]) for i in np.nonzero(sizes == 16)[0]])
    h2 = nd.h[0] ** 2
    E = np.abs(w2.cpu().numpy()[pos] - wo[0][pos]).max() * h2 / max(1.0, np.abs(wo[0][pos]).max() * h2)
    assert E <= 1e-10


def test_zero_network_rejected_at_default_tolerances(gpu):
    """The acceptance test judges what the network controls: the zero network's
    output needs a correction of the whole weights (ratio 1 > 0.25), so at the
    default tolerances every stencil falls back to the plain solve, bit for bit;
    a tolerance above 1 accepts them all."""
    nd, off, X, od, idx = _plain_and_stencils(gpu)
    wp, _ = rb.compute_weights(X, od, idx, 15, 2, ("lap",), precision="f64")
    rb.surrogate_load(torch.zeros(rb.MLP_NPARAM, dtype=torch.float32, device=gpu))
    w, st = rb.surrogate_weights(X, od, idx, 15)
    assert torch.all(st == rb.ST_SURROGATE_REJECTED)
    assert torch.equal(w, wp[0])
    # its correction ratio is exactly 1: a tolerance just above 1 accepts every stencil
    _, st2 = rb.surrogate_weights(X, od, idx, 15, surrogate_corr_tol=1.0 + 1e-12)
    assert torch.all(st2 == rb.ST_SURROGATE)


def test_zero_network_is_min_norm_projection(gpu):
    nd, off, X, od, idx = _plain_and_stencils(gpu)
    zero = torch.zeros(rb.MLP_NPARAM, dtype=torch.float32, device=gpu)
    rb.surrogate_load(zero)
    w, st = rb.surrogate_weights(X, od, idx, 15, surrogate_tol=1e300, surrogate_corr_tol=1e300)
    idx_n = idx.cpu().numpy().reshape(-1, 15)
    Xh = nd.X[idx_n] - nd.X[idx_n[:, :1]]
    s = np.sqrt((Xh ** 2).sum(-1)).max(1)
    wo, _ = oproj.project(np.zeros((nd.N, 15)), Xh / s[:, None, None], 2, oproj.lap_lq(2, 2))
    wo = (wo / (s * s)[:, None]).reshape(-1)
    h2 = nd.h[0] ** 2
    assert np.abs(w.cpu().numpy() - wo).max() * h2 / max(1.0, np.abs(wo).max() * h2) <= 1e-10


def test_training_gain_and_resume(gpu, tmp_path):
    """Train on 40 seeded disks (~80k stencils).  On the held-out disk (seed 1001) the
    operators are used in the manufactured Poisson problem -lap u = f, u = u_0 on the
    boundary (u_0 = sin(pi x) sin(pi y)): the trained network's projected weights must
    solve it about as well as the plain weights, where the zero network (projection
    alone: the minimum-norm consistent weights) gives an unstable operator.  The
    pointwise Laplacian error e_h of all three is reported."""
    import time
    torch.manual_seed(0)
    data = S.build_training_set(S.training_node_sets(40), device=gpu)
    assert torch.isfinite(data.feat).all() and torch.isfinite(data.target).all()
    # checkpoint / resume: a saved and reloaded state continues with the same bits
    a = S.TrainState.init(21, device=gpu)
    S.train(a, data, epochs=1, batch=4096, lr=1e-3, seed=3, total_steps=40)
    ck = str(tmp_path / "ck.pt")
    a.save(ck)
    b = S.TrainState.load(ck, device=gpu)
    assert torch.equal(b.params, a.params) and torch.equal(b.m, a.m) and torch.equal(b.v, a.v) and b.step == a.step
    assert torch.equal(b.packed, a.packed)
    S.train(a, data, epochs=1, batch=4096, lr=1e-3, seed=5, total_steps=40)
    S.train(b, data, epochs=1, batch=4096, lr=1e-3, seed=5, total_steps=40)
    assert torch.equal(a.params, b.params)
    # training
    st = S.TrainState.init(22, device=gpu)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = S.train(st, data, epochs=60, batch=1024, lr=1e-3, seed=4)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"  {st.step} steps in {dt:.2f} s; loss {hist[0]:.3e} -> {hist[-1]:.3e}", flush=True)
    assert hist[-1] < 0.1 * hist[0]

    nd, off, X, od, idx = _plain_and_stencils(gpu)
    wp, _ = rb.compute_weights(X, od, idx, 15, 2, ("lap",), precision="f64")
    wt, stt = S.surrogate_laplacian(X, od, idx, st.params)
    # the ablation: the zero network's projection alone (the correction gate would reject it all)
    wz, stz = S.surrogate_laplacian(X, od, idx, torch.zeros_like(st.params), corr_tol=float("inf"))
    idx_n = idx.cpu().numpy()
    interior = ~nd.is_boundary
    e, pe = {}, {}
    for name, w in (("plain", wp[0]), ("trained", wt), ("zero", wz)):
        wv = w.cpu().numpy()
        approx = (wv * opoi.u0(nd.X)[idx_n]).reshape(-1, 15).sum(1)
        e[name] = float(np.abs(approx - opoi.lap_u0(nd.X))[interior].max())
        pe[name] = opoi.solve_dirichlet(nd.X, nd.is_boundary, off, idx_n, wv)[1]
    acc = float((stt.cpu().numpy() == rb.ST_SURROGATE).mean())
    wpn = wp[0].cpu().numpy().reshape(-1, 15)
    dev_t = np.abs(wt.cpu().numpy().reshape(-1, 15) - wpn).max(1) / np.abs(wpn).max(1)
    dev_z = np.abs(wz.cpu().numpy().reshape(-1, 15) - wpn).max(1) / np.abs(wpn).max(1)
    print(f"  Poisson max error: plain {pe['plain']:.3e}  trained {pe['trained']:.3e}  zero network {pe['zero']:.3e}",
          flush=True)
    print(f"  e_h: plain {e['plain']:.3e}  trained {e['trained']:.3e}  zero network {e['zero']:.3e}; accepted {acc:.3f}",
          flush=True)
    print(f"  per-stencil max|w - w_plain| / max|w_plain|: trained median {np.median(dev_t):.2e} "
          f"max {dev_t.max():.2e}; zero network median {np.median(dev_z):.2e}", flush=True)
    assert acc >= 0.9
    assert pe["trained"] <= 3.0 * pe["plain"]
    assert pe["zero"] >= 1e3 * pe["trained"]
    assert np.median(dev_t) < 0.2 * np.median(dev_z)
