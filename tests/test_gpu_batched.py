"""GPU parity of the batched persistent form (mixed dimension, per-node degree and
stencil size, one launch) and of large systems (n + m up to 128), against the oracle."""
import numpy as np
import pytest
import torch

import nodesets as ns
import paper_1912_13282_amd as rb
from oracle import knn as oknn
from oracle import rbffd as orbf

pytestmark = pytest.mark.gpu

ORD = {"lap": 2, "dx": 1, "dy": 1, "dz": 1}


def scaled_err(wg, wo, ops, off, h):
    hn = np.repeat(h, np.diff(off))
    worst = 0.0
    for r, op in enumerate(ops):
        sc = hn ** ORD[op]
        den = max(1.0, float(np.max(np.abs(wo[r]) * sc)))
        worst = max(worst, float(np.max(np.abs(wg[r] - wo[r]) * sc)) / den)
    return worst


def build_batch(dev, per_domain=1500, seed=1003):
    """The four mixed-batch domains at a reduced size (same recipe as the 8M-node batch)."""
    doms, ref = [], []
    for nd, P, n in ns.mixed_domains(per_domain, seed):
        off = ns.offsets_from_sizes(n)
        Xd = torch.from_numpy(nd.X).to(dev)
        od = torch.from_numpy(off).to(dev)
        idx = rb.select_stencils(Xd, od, int(n.max()))
        ops = ("lap", "dx", "dy") + (("dz",) if nd.d == 3 else ())
        D = rb.Domain(Xd, od, idx, int(n.max()), torch.from_numpy(P).to(dev), ops)
        doms.append(D)
        ref.append((nd, P, off, ops))
    torch.cuda.synchronize()
    return doms, ref


@pytest.mark.parametrize("precision", ["f64", "f32_ir"])
def test_batched_mixed_parity(gpu, precision):
    doms, ref = build_batch(gpu)
    rb.compute_weights_batched(doms, precision=precision)
    torch.cuda.synchronize()
    for D, (nd, P, off, ops) in zip(doms, ref):
        idx = D.idx.cpu().numpy()
        o2, i2 = oknn.knn_exact(nd.X, np.diff(off))
        assert np.array_equal(idx, i2), nd.meta["domain"]
        wo, sto = orbf.weights(nd.X, off, idx, P.astype(np.int64), ops)
        st = D.status.cpu().numpy()
        assert sto.min() == 0
        if precision == "f64":
            assert np.all(st == 0), np.unique(st, return_counts=True)
            tol = 1e-10
        else:
            assert np.all((st == 1) | (st == 2)), np.unique(st, return_counts=True)
            tol = 1e-9
        E = scaled_err(D.w.cpu().numpy(), wo, ops, off, nd.h)
        print(f"  {nd.meta['domain']} {precision} E = {E:.2e} status {np.unique(st, return_counts=True)}", flush=True)
        assert E <= tol


@pytest.mark.parametrize("precision", ["f64", "f32_ir"])
def test_autotune_plan_and_cache(gpu, tmp_path, precision):
    """Per-class plans: every class gets its own tuned (chunk, waves per CU); the
    cache serves the same plans for the same signature (and not for other solver
    options); plans change the scheduling, never the results (bit-identical)."""
    doms, ref = build_batch(gpu, per_domain=600)
    cache = str(tmp_path / "plans.txt")
    plans = rb.autotune_batched(doms, precision=precision, cache_path=cache)
    assert len(plans) == len(rb.batched_class_sizes())
    assert all(p["chunk"] >= 1 and p["waves_per_cu"] >= 1 for p in plans)
    assert rb.get_plan() == [{"chunk": p["chunk"], "waves_per_cu": p["waves_per_cu"]} for p in plans]
    w1 = [D.w.clone() for D in doms]
    s1 = [D.status.clone() for D in doms]
    rb.set_plan(None)
    plans2 = rb.autotune_batched(doms, precision=precision, cache_path=cache)   # served from the cache
    assert [(p["chunk"], p["waves_per_cu"]) for p in plans2] == [(p["chunk"], p["waves_per_cu"]) for p in plans]
    assert len(open(cache).read().splitlines()) == 1
    rb.autotune_batched(doms, precision=precision, cache_path=cache, phs_power=5)   # other options: tuned again
    assert len(open(cache).read().splitlines()) == 2
    for plan in (plans2, (1, 4), (16, 16), [(1 + c % 5, 4 + 4 * (c % 4)) for c in range(len(plans))]):
        rb.set_plan(plan)
        rb.compute_weights_batched(doms, precision=precision)
        for a, b, D in zip(w1, s1, doms):
            assert torch.equal(a, D.w) and torch.equal(b, D.status)   # plans change scheduling, never results
    rb.set_plan(None)


@pytest.mark.parametrize("precision", ["f64", "f32_ir"])
def test_large_systems_parity(gpu, precision):
    """n = 65, degree 4 in 3D (m = 35, n + m = 100): the large-3D workload's stencil shape."""
    C, R = ns.random_balls(1005, count=8)
    nd = ns.cube_minus_balls(1.0 / 14, 1006, C, R)
    off = ns.offsets_from_sizes(np.full(nd.N, 65, np.int64))
    Xd, od = torch.from_numpy(nd.X).to(gpu), torch.from_numpy(off).to(gpu)
    idx = rb.select_stencils(Xd, od, 65)
    ops = ("lap", "dx", "dy", "dz")
    w, st = rb.compute_weights(Xd, od, idx, 65, 4, ops, precision=precision)
    torch.cuda.synchronize()
    idx = idx.cpu().numpy()
    o2, i2 = oknn.knn_exact(nd.X, 65)
    assert np.array_equal(idx, i2)
    wo, sto = orbf.weights(nd.X, off, idx, 4, ops)
    st = st.cpu().numpy()
    if precision == "f64":
        assert np.all(st == rb.ST_OK)
    else:
        # float32 elimination (two rows per lane) + float64 refinement; FALLBACK is allowed
        # per stencil but the refined form must carry the workload
        assert np.all((st == rb.ST_REFINED) | (st == rb.ST_FALLBACK))
        print(f"  refined fraction {np.mean(st == rb.ST_REFINED):.4f}", flush=True)
        assert np.mean(st == rb.ST_REFINED) >= 0.99
    E = scaled_err(w.cpu().numpy(), wo, ops, off, nd.h)
    print(f"  N={nd.N} E={E:.2e}", flush=True)
    assert E <= (1e-10 if precision == "f64" else 1e-9)


def test_large_ir_forced_fallback_equals_f64(gpu):
    """max_refine = 0 sends every stencil of the refined large-system form to the
    float64 four-wave solve: the weights equal the plain float64 call bit for bit."""
    C, R = ns.random_balls(1005, count=8)
    nd = ns.cube_minus_balls(1.0 / 12, 1006, C, R)
    off = ns.offsets_from_sizes(np.full(nd.N, 65, np.int64))
    Xd, od = torch.from_numpy(nd.X).to(gpu), torch.from_numpy(off).to(gpu)
    idx = rb.select_stencils(Xd, od, 65)
    ops = ("lap", "dx", "dy", "dz")
    w64, _ = rb.compute_weights(Xd, od, idx, 65, 4, ops, precision="f64")
    wir, st = rb.compute_weights(Xd, od, idx, 65, 4, ops, precision="f32_ir", max_refine=0)
    assert torch.all(st == rb.ST_FALLBACK)
    assert torch.equal(w64, wir)


@pytest.mark.parametrize("precision", ["f64", "f32_ir"])
@pytest.mark.parametrize("n,P", [(59, 2), (70, 2), (89, 4), (91, 4), (113, 4)])
def test_large_systems_sizes_2d(gpu, n, P, precision):
    """2D systems of 65, 76, 104, 106 and 128 unknowns (size classes 80, 100, 108 and
    128 above 64; the refined form reaches 108 unknowns, beyond that it reports FALLBACK)."""
    nd = ns.disk(0.07, 1007)
    off = ns.offsets_from_sizes(np.full(nd.N, n, np.int64))
    Xd, od = torch.from_numpy(nd.X).to(gpu), torch.from_numpy(off).to(gpu)
    idx = rb.select_stencils(Xd, od, n)
    ops = ("lap", "dx", "dy")
    w, st = rb.compute_weights(Xd, od, idx, n, P, ops, precision=precision)
    torch.cuda.synchronize()
    wo, sto = orbf.weights(nd.X, off, idx.cpu().numpy(), P, ops)
    st = st.cpu().numpy()
    good = np.nonzero(sto == 0)[0]
    M = n + (6 if P == 2 else 15)
    if precision == "f64":
        assert good.size >= 0.99 * nd.N and np.all(st[good] == rb.ST_OK)
    elif M <= 108:
        assert good.size >= 0.99 * nd.N and np.all((st[good] == rb.ST_REFINED) | (st[good] == rb.ST_FALLBACK))
        assert np.mean(st[good] == rb.ST_REFINED) >= 0.95
    else:
        assert good.size >= 0.99 * nd.N and np.all(st[good] == rb.ST_FALLBACK)
    pos = np.concatenate([np.arange(off[i], off[i + 1]) for i in good])
    offg = ns.offsets_from_sizes(np.full(good.size, n, np.int64))
    E = scaled_err(w.cpu().numpy()[:, pos], wo[:, pos], ops, offg, nd.h[good])
    print(f"  N={nd.N} M={M} {precision} E={E:.2e}", flush=True)
    assert E <= (1e-10 if precision == "f64" else 1e-9)


@pytest.mark.parametrize("P", [0, 1, 2, 4])
def test_batched_uniform_degree_matches_per_call(gpu, P):
    """Domains with a uniform degree (no per-node array), 2D and 3D in one batch: the
    batched weights equal the per-call weights and the oracle."""
    nd2 = ns.disk(0.05, 1011)
    nd3 = ns.cube_minus_sphere(1.0 / 12, 1012)
    doms, ref = [], []
    for nd, n0 in ((nd2, 14), (nd3, 30)):
        n = max(n0, -(-3 * ns.n_monomials(nd.d, P) // 2))  # at least 1.5 m (3D degree 4: 53 + 35 unknowns)
        off = ns.offsets_from_sizes(np.full(nd.N, n, np.int64))
        Xd, od = torch.from_numpy(nd.X).to(gpu), torch.from_numpy(off).to(gpu)
        idx = rb.select_stencils(Xd, od, n)
        ops = ("lap", "dx", "dy") + (("dz",) if nd.d == 3 else ())
        doms.append(rb.Domain(Xd, od, idx, n, P, ops))
        w1, s1 = rb.compute_weights(Xd, od, idx, n, P, ops, precision="f64")
        ref.append((nd, off, ops, w1, s1))
    rb.compute_weights_batched(doms, precision="f64")
    torch.cuda.synchronize()
    for D, (nd, off, ops, w1, s1) in zip(doms, ref):
        st = D.status.cpu().numpy()
        assert np.array_equal(st, s1.cpu().numpy())
        wo, sto = orbf.weights(nd.X, off, D.idx.cpu().numpy(), P, ops)
        good = np.nonzero((st == 0) & (sto == 0))[0]
        assert good.size >= 0.9 * nd.N
        pos = np.concatenate([np.arange(off[i], off[i + 1]) for i in good])
        offg = ns.offsets_from_sizes(np.diff(off)[good])
        E = scaled_err(D.w.cpu().numpy()[:, pos], wo[:, pos], ops, offg, nd.h[good])
        E1 = scaled_err(D.w.cpu().numpy()[:, pos], w1.cpu().numpy()[:, pos], ops, offg, nd.h[good])
        print(f"  d={nd.d} P={P}: vs oracle {E:.1e}, vs per-call {E1:.1e}", flush=True)
        assert E <= 1e-10 and E1 <= 1e-12


def test_batched_phs5(gpu):
    doms, ref = build_batch(gpu, per_domain=500)
    rb.compute_weights_batched(doms, precision="f64", phs_power=5)
    torch.cuda.synchronize()
    for D, (nd, P, off, ops) in zip(doms, ref):
        wo, sto = orbf.weights(nd.X, off, D.idx.cpu().numpy(), P.astype(np.int64), ops, phs_power=5)
        st = D.status.cpu().numpy()
        good = np.nonzero((st == 0) & (sto == 0))[0]
        assert good.size >= 0.98 * nd.N
        pos = np.concatenate([np.arange(off[i], off[i + 1]) for i in good])
        offg = ns.offsets_from_sizes(np.diff(off)[good])
        E = scaled_err(D.w.cpu().numpy()[:, pos], wo[:, pos], ops, offg, nd.h[good])
        print(f"  {nd.meta['domain']} r^5: E = {E:.1e}", flush=True)
        assert E <= 1e-10
