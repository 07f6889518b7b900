"""Benchmark of the RBF-FD stencil hot path on one MI355X.

Default workload (cube_sphere3d): [0,1]^3 minus the ball B((1/2,1/2,1/2), 0.3),
jittered lattice h = 1/106 plus face lattice and Fibonacci sphere nodes
(1,096,553 nodes), n = 35, degree 3 (m = 20), operators Laplacian, d/dx, d/dy,
d/dz.  One step = rbf_select_stencils + rbf_compute_weights + rbf_assemble_csr
over the whole node set, inputs resident in HBM.  The reported form is FP32 LU +
FP64 refinement; the plain FP64 form is timed beside it on the same inputs.

Other workloads (the same JSON contract, one line each):
  mixed    four 2D/3D domains (disk with holes, L-shape, cube minus sphere,
           torus), 2M nodes each, per-node degree 2-4 and n in [12, 70]; the
           weights of all four in one persistent launch per precision, plan
           chosen by the autotuner before the timed steps
  learned  the learned Laplacian surrogate: trained on the GPU on 5,000 seeded
           disk node sets (10M stencils), timed on a 1.7M-node disk against the
           plain FP64 and FP32+refinement solves; quality on the 2,007-node disk
  large3d  [0,1]^3 minus 64 random balls, h = 1/256 (about 16M nodes), n = 65,
           degree 4 (n + m = 100), with CSR
  poisson3d / poisson2d
           the benchmark problem of Sec. 5: -lap u = f on the annulus B(0,1)
           minus B(0,1/2), u_0 = prod sin(pi x_a) on the boundary, n = 35 (3D) or
           9 (2D), degree 2, about 1M nodes; stencils, weights, implicit
           assembly and BiCGStab (Jacobi scaling, tol 1e-10) per step
  wls      the GWLS engine (Sec. 2.2.1) on the default node set: monomials of degree
           3, Gaussian weight (sigma 1 on the scaled offsets), four operators, with
           kNN and CSR
  counters one launch of each hot kernel at its workload's shape, for rocprofv3
           counter passes: stencils + FP64 + FP32-refined weights + CSR of the
           default node set, both solvers above 64 unknowns on a 1M-node copy of
           large3d, the batched form of a 200k-per-domain mixed batch, the
           surrogate on a 1.7M-node disk, and a 1 GiB copy (byte calibration)
  explicit explicit Euler steps of du/dt = lap u + 5 on the default node set
           (faces u = x, sphere zero flux), each followed by the evaluation of
           the four operators on the new field; weights computed beforehand

    python bench.py [--workload W] [--steps K] [--warmup W] [--no-cpu] ...

Prints one JSON line.  Only one GPU is supported: --gpus N with N > 1 exits.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RBF-FD stencils/s (kNN+weights) mixed/learned vs plain FP64 at stated error"
PEAK_FP64_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (FMA, one lane op per clock)
PEAK_BF16_TFLOPS = 2500.0   # dense bf16 MFMA
PEAK_HBM_GBS = 8000.0
ORD = {"lap": 2, "dx": 1, "dy": 1, "dz": 1}

# HBM traffic of each workload's dominant kernel, from FETCH_SIZE / WRITE_SIZE
# passes recorded under profiles/; valid while that kernel's sources hash to the
# recorded value.
CSRC = "paper_1912_13282_amd/csrc/"
TRAFFIC = {
    "cube_sphere3d": ("profiles/traffic_weights_cube_minus_sphere_3d.txt",
                      [CSRC + f for f in ("common.hpp", "wsolve.hpp", "wsolve_pair.hpp", "weights_kernels.hpp",
                                          "weights.hip", "wcls_56.hip")]),
    "explicit": ("profiles/traffic_apply_explicit_heat_cube_minus_sphere_3d.txt",
                 [CSRC + f for f in ("common.hpp", "rowdot.hpp", "apply.hip")]),
    "poisson3d": ("profiles/traffic_bicgstab_block_jacobi_poisson_annulus_3d.txt",
                  [CSRC + f for f in ("common.hpp", "rowdot.hpp", "cellorder.hpp", "implicit.hip")]),
}


def weights_flops(n, m, d, R):
    """Algorithmic FLOPs of one stencil's weights: LU of the (n+m)^2 system,
    forward/back substitution of R right-hand sides, and the n^2 RBF entries
    (d differences, d squares, d-1 additions, a square root and a product)."""
    M = n + m
    return (2.0 / 3.0) * M ** 3 + 2.0 * R * M * M + (3 * d + 1) * n * n


def knn_bytes(n, d):
    """Algorithmic HBM bytes of stencil selection: read the node, write n indices."""
    return 8.0 * d + 4.0 * n


def csr_bytes(n, R):
    """Read idx and w, write col and vals, plus the row pointer."""
    return 2.0 * (4.0 * n + 8.0 * R * n) + 8.0


SURROGATE_FLOPS = 2.0 * (32 * 128 + 128 * 128 * 2 + 128 * 16)   # MFMA work per stencil (padded shapes)
SURROGATE_BYTES = 8 + 15 * 4 + 15 * 8 + 1 + 16                  # offsets, idx, w, status, centre coordinates


def source_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload: str, form: str | None = None):
    """HBM bytes per launch of the workload's dominant kernel from the committed
    FETCH_SIZE / WRITE_SIZE passes, or None if absent or taken on other sources."""
    if workload not in TRAFFIC:
        return None
    path, files = TRAFFIC[workload]
    path = os.path.join(ROOT, path)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != source_hash(files) or (form is not None and kv.get("form") != form):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cube_sphere3d", choices=["cube_sphere3d", "mixed", "learned", "large3d", "explicit", "poisson3d", "poisson2d", "wls",
                             "counters"])
    ap.add_argument("--form", default="f32_ir", choices=["f32_ir", "f64"])
    ap.add_argument("--precond", default="auto", choices=["auto", "block_jacobi", "jacobi", "none"],
                    help="poisson: BiCGStab preconditioner (auto: block-Jacobi in 3D, Jacobi in 2D)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-compare", action="store_true", help="time only the reported form")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="nodes in the CPU oracle sample (default: about 10 s of oracle work per workload)")
    ap.add_argument("--per-domain", type=int, default=2_000_000, help="mixed: nodes per domain")
    ap.add_argument("--tune-per-domain", type=int, default=200_000, help="mixed: nodes per domain of the tuning batch")
    ap.add_argument("--train-sets", type=int, default=5000, help="learned: training node sets (2,008 nodes each)")
    ap.add_argument("--train-epochs", type=int, default=8)
    ap.add_argument("--no-legs", action="store_true",
                    help="default workload: skip the compact legs of the 16M-node large-3D and the 8M-stencil "
                         "mixed workloads")
    ap.add_argument("--err-sample", type=int, default=0,
                    help="with --no-cpu: weights error against the oracle on this many sampled stencils "
                         "(oracle weights of the GPU's stencils)")
    ap.add_argument("--batched-forms", action="store_true",
                    help="large3d / cube_sphere3d: also time the batched persistent form (both precisions)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed steps, run a plain 1 GiB read + 1 GiB write elementwise kernel "
                         "(torch.neg on float64) three times, the reference for HBM byte counters")
    return ap.parse_args()


class Timer:
    """HIP events on the current stream (the stream every library call is enqueued on)."""

    def __init__(self, torch, phases):
        self.torch, self.phases = torch, phases
        self.stream = torch.cuda.current_stream()

    def run(self, step, K, W):
        torch = self.torch
        for _ in range(W):
            step(None)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(self.phases) + 1)] for _ in range(K)]
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        wall = time.perf_counter()
        t0.record(self.stream)
        for k in range(K):
            step(evs[k])
        t1.record(self.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall
        ph = np.array([[e[j].elapsed_time(e[j + 1]) for j in range(len(self.phases))] for e in evs])
        return t0.elapsed_time(t1) / K, 1000.0 * wall / K, dict(zip(self.phases, ph.mean(axis=0).tolist()))


def scaled_err(wg, wo, ops, hn):
    worst = 0.0
    for c, op in enumerate(ops):
        sc = hn ** ORD[op]
        den = max(1.0, float(np.max(np.abs(wo[c]) * sc)))
        worst = max(worst, float(np.max(np.abs(wg[c] - wo[c]) * sc)) / den)
    return worst


def draw_sample(N, sample_size, seed=12345):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(N, size=min(sample_size, N), replace=False))


def sample_positions(off, sample):
    return np.concatenate([np.arange(off[i], off[i + 1]) for i in sample])


def cpu_oracle(X, sizes, P, ops, sample):
    """The oracle, untuned: exact kNN (k-d tree + exact re-rank, against all nodes)
    and weights (one LAPACK gesv per stencil) on a seeded sample, BLAS limited to
    one thread.  Returns (baseline dict, sample offsets, idx, W)."""
    from threadpoolctl import threadpool_limits

    from oracle import knn as oknn
    from oracle import rbffd as orbf

    N = X.shape[0]
    Ps = np.broadcast_to(np.asarray(P), (N,))[sample]
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        c0 = time.process_time()
        soff, sidx = oknn.knn_exact(X, sizes, nodes=sample)
        Wo, sto = orbf.weights(X, soff, sidx, Ps, ops)
        dt = time.perf_counter() - t
        cpu_s = time.process_time() - c0
    threads = max(1, int(round(cpu_s / dt)))   # threads the oracle kept busy on average
    base = {"value": sample.size / dt, "unit": "stencils/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample.size} seeded random nodes of the same workload (kNN against all {N} nodes + weights), "
                      f"{dt:.1f} s wall, {cpu_s:.1f} s CPU, BLAS limited to one thread"}
    return base, soff, sidx, Wo


_POOL_ARGS = None


def _oracle_chunk(nodes):
    """Worker of cpu_oracle_all_cores: the oracle on its share of the sample (one
    BLAS thread; the node array arrives through fork)."""
    from threadpoolctl import threadpool_limits

    from oracle import knn as oknn
    from oracle import rbffd as orbf
    X, sizes, P, ops = _POOL_ARGS
    with threadpool_limits(limits=1):
        soff, sidx = oknn.knn_exact(X, sizes, nodes=nodes)
        orbf.weights(X, soff, sidx, np.broadcast_to(np.asarray(P), (X.shape[0],))[nodes], ops)
    return nodes.size


def cpu_oracle_all_cores(X, sizes, P, ops, sample, max_workers=16):
    """The same oracle on every host core the process may use (a fork pool over
    os.sched_getaffinity, at most max_workers), one BLAS thread per worker; each
    worker builds its own k-d tree.  Returns the baseline dict."""
    import multiprocessing as mp
    global _POOL_ARGS
    cores = min(len(os.sched_getaffinity(0)), max_workers)
    _POOL_ARGS = (X, sizes, P, ops)
    parts = [np.ascontiguousarray(c) for c in np.array_split(sample, cores * 4) if c.size]
    t = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        done = sum(pool.map(_oracle_chunk, parts, chunksize=1))
    dt = time.perf_counter() - t
    _POOL_ARGS = None
    return {"value": done / dt, "unit": "stencils/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} seeded random nodes (kNN against all {X.shape[0]} nodes + weights) over a pool of "
                      f"{cores} processes (os.sched_getaffinity, one BLAS thread each, tree built per process), "
                      f"{dt:.1f} s wall"}


def sample_errors(snap, sample, soff, sidx, Wo, ops, hn_sample):
    """Scaled max error of each GPU form on the oracle sample, and stencil equality.
    snap[form] = (weights at the sample positions [R, P], indices there or None)."""
    err = {}
    hn = np.repeat(hn_sample, np.diff(soff))
    for f, (wg, ig) in snap.items():
        if wg is not None:
            err[f] = {"scaled_max_err": scaled_err(wg, Wo, ops, hn),
                      "tolerance": 1e-10 if f == "f64" else 1e-9, "sample": int(sample.size)}
        if ig is not None:
            err["stencils_bit_exact_on_sample"] = bool(np.array_equal(ig, sidx))
    return err


def calib_copy(torch, dev):
    src = torch.randn(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(f"[bench] calibration copy: 3 x (read {src.numel() * 8} B + write {dst.numel() * 8} B)",
          file=sys.stderr, flush=True)


def base_line(a, value, ms, dtype, config):
    return {"metric": METRIC, "value": value, "unit": "stencils/s", "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def status_counts(st):
    return {int(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))}


# ---------------------------------------------------------------- cube_sphere3d / large3d
def bench_uniform(a, torch, rb, B, name):
    import nodesets as ns
    dev = torch.device("cuda:0")
    t = time.perf_counter()
    wl = ns.workload(name)
    nd = wl["nodes"][0]
    print(f"[bench] {name}: {nd.N} nodes generated in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    n, P, ops = wl["n"], wl["P"], wl["ops"]
    d = nd.d
    m = math.comb(P + d, d)
    R = len(ops)
    N = nd.N
    off = ns.offsets_from_sizes(np.full(N, n, dtype=np.int64))
    nnz = int(off[-1])
    X = torch.from_numpy(nd.X).to(dev)
    offsets = torch.from_numpy(off).to(dev)
    idx = torch.empty(nnz, dtype=torch.int32, device=dev)
    ws = torch.empty(B.select_stencils_workspace(N, d, n), dtype=torch.uint8, device=dev)
    w = torch.empty((R, nnz), dtype=torch.float64, device=dev)
    status = torch.empty(N, dtype=torch.int8, device=dev)
    row_ptr = torch.empty(N + 1, dtype=torch.int64, device=dev)
    col = torch.empty(nnz, dtype=torch.int32, device=dev)
    vals = torch.empty((R, nnz), dtype=torch.float64, device=dev)
    ctx = rb.context(dev)
    timer = Timer(torch, ["select_stencils", "compute_weights", "assemble_csr"])
    sample = draw_sample(N, a.cpu_sample or 150_000)
    pos_t = torch.from_numpy(sample_positions(off, sample)).to(dev)

    def make_step(form):
        def step(e):
            if e:
                e[0].record(timer.stream)
            rb.select_stencils(X, offsets, n, idx=idx, workspace=ws, ctx=ctx)
            if e:
                e[1].record(timer.stream)
            rb.compute_weights(X, offsets, idx, n, P, ops, precision=form, w=w, status=status, ctx=ctx)
            if e:
                e[2].record(timer.stream)
            rb.assemble_csr(offsets, idx, w, n, row_ptr=row_ptr, col=col, vals=vals, ctx=ctx)
            if e:
                e[3].record(timer.stream)
        return step

    if a.no_cpu and a.err_sample:
        sample = draw_sample(N, a.err_sample)
        pos_t = torch.from_numpy(sample_positions(off, sample)).to(dev)

    # the batched persistent form on the same node set: one domain, its plan tuned
    # per precision on a coarser copy of the workload (about 1M nodes)
    dom, wsb, bplans = None, None, {}
    if a.batched_forms:
        dom = rb.Domain(X, offsets, idx, n, P, ops)
        dom.w, dom.status = w, status          # the same output buffers as the per-call form
        wsb = torch.empty(B.batched_workspace([dom]), dtype=torch.uint8, device=dev)
        tw = ns.workload(name, h=(1.0 / 100 if name == "large3d" else 1.0 / 60))
        tnd = tw["nodes"][0]
        toff = torch.from_numpy(ns.offsets_from_sizes(np.full(tnd.N, n, dtype=np.int64))).to(dev)
        tX = torch.from_numpy(tnd.X).to(dev)
        tdom = rb.Domain(tX, toff, rb.select_stencils(tX, toff, n, ctx=ctx), n, P, ops)
        for f in ("f32_ir", "f64"):
            t = time.perf_counter()
            bplans[f] = rb.autotune_batched([tdom], precision=f, ctx=ctx)
            print(f"[bench] {name} batched {f}: plans tuned on {tnd.N} stencils in {time.perf_counter() - t:.1f} s",
                  file=sys.stderr, flush=True)
        del tdom, tX, toff

    def make_batched_step(form):
        def step(e):
            if e:
                e[0].record(timer.stream)
            rb.select_stencils(X, offsets, n, idx=idx, workspace=ws, ctx=ctx)
            if e:
                e[1].record(timer.stream)
            rb.compute_weights_batched([dom], precision=form, workspace=wsb, ctx=ctx)
            if e:
                e[2].record(timer.stream)
            rb.assemble_csr(offsets, idx, w, n, row_ptr=row_ptr, col=col, vals=vals, ctx=ctx)
            if e:
                e[3].record(timer.stream)
        return step

    results, snap = {}, {}
    forms = [a.form] if a.no_compare else [a.form] + [f for f in ("f64", "f32_ir") if f != a.form]
    if a.batched_forms:
        forms += ["batched_f32_ir", "batched_f64"]
    for f in forms:
        if f.startswith("batched_"):
            rb.set_plan(bplans[f[8:]], ctx=ctx)
            ms, wall, ph = timer.run(make_batched_step(f[8:]), a.steps, a.warmup)
        else:
            ms, wall, ph = timer.run(make_step(f), a.steps, a.warmup)
        st = status.cpu().numpy()
        results[f] = dict(form=f, ms_per_step=ms, wall_ms_per_step=wall, phases_ms=ph,
                          stencils_per_s=N / (ms / 1e3),
                          knn_weights_stencils_per_s=N / ((ph["select_stencils"] + ph["compute_weights"]) / 1e3),
                          status_counts=status_counts(st), fallback_fraction=float(np.mean(st == rb.ST_FALLBACK)))
        if not a.no_cpu or a.err_sample:
            snap[f] = (w[:, pos_t].cpu().numpy(), idx[pos_t].cpu().numpy() if f == forms[0] else None)
        print(f"[bench] {name} {f}: {ms:.3f} ms/step  phases {ph}", file=sys.stderr, flush=True)
    rb.set_plan(None, ctx=ctx)

    main = results[a.form]
    flop = weights_flops(n, m, d, R)
    achieved = flop * N / (main["phases_ms"]["compute_weights"] / 1e3) / 1e12
    M = n + m
    if M > 64:
        kernel = ("k_weights_ir_pair<100> + k_weights_quad<100> (fallback pass)" if a.form == "f32_ir"
                  else "k_weights_quad<100>")
    elif a.form == "f32_ir":
        kernel = "k_weights_ir<56> + k_weights_f64<56> (fallback pass)"
    else:
        kernel = "k_weights_f64<56>"
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS,
                "traffic": recorded_traffic(name, a.form),
                "kernel": kernel, "flop_per_stencil": flop, "stencils_per_launch": N}
    phases_roofline = {}
    for ph_name, per in (("select_stencils", knn_bytes(n, d)), ("assemble_csr", csr_bytes(n, R))):
        gbs = per * N / (main["phases_ms"][ph_name] / 1e3) / 1e9
        phases_roofline[ph_name] = {"bound": "hbm", "bytes_per_stencil": per, "achieved_GBs": gbs,
                                    "frac": gbs / PEAK_HBM_GBS}
    label = {"cube_sphere3d": "cube_minus_sphere_3d", "large3d": "cube_minus_64_balls_3d"}[name]
    out = base_line(a, main["stencils_per_s"], main["ms_per_step"], "f32+f64" if a.form == "f32_ir" else "f64",
                    {"workload": label, "N": N, "nnz": nnz, "n": n, "degree": P, "m": m, "ops": list(ops),
                     "phs_power": 3, "form": a.form, "step": "select_stencils + compute_weights + assemble_csr"})
    out.update(roofline=roofline, phases_roofline=phases_roofline, forms=results)
    if "f64" in results and "f32_ir" in results:
        out["mixed_vs_f64"] = (results["f32_ir"]["knn_weights_stencils_per_s"] /
                               results["f64"]["knn_weights_stencils_per_s"])
    if a.calib_copy:
        calib_copy(torch, dev)
    if not a.no_cpu:
        base, soff, sidx, Wo = cpu_oracle(nd.X, n, P, ops, sample)
        out["cpu_baseline"] = base
        out["error"] = sample_errors(snap, sample, soff, sidx, Wo, ops, nd.h[sample])
        if name == "cube_sphere3d":
            out["cpu_baseline_all_cores"] = cpu_oracle_all_cores(nd.X, n, P, ops, draw_sample(N, N, seed=777))
    elif a.err_sample:
        from oracle import rbffd as orbf
        ig = snap[forms[0]][1]
        soff = ns.offsets_from_sizes(np.full(sample.size, n, dtype=np.int64))
        Wo, _ = orbf.weights(nd.X, soff, ig, P, ops)
        err = sample_errors({f: (v[0], None) for f, v in snap.items()}, sample, soff, ig, Wo, ops, nd.h[sample])
        for f in err:
            err[f]["tolerance"] = 1e-10 if f.endswith("f64") else 1e-9
        err["note"] = "oracle weights of the GPU's stencils (the stencils are checked against the oracle in the tests)"
        out["error"] = err
    return out


# ---------------------------------------------------------------- mixed batch
def bench_mixed(a, torch, rb, B):
    import nodesets as ns
    dev = torch.device("cuda:0")
    t = time.perf_counter()
    parts = ns.mixed_domains(a.per_domain)
    print(f"[bench] mixed: nodes generated in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    ctx = rb.context(dev)
    doms, meta, flop_total, N_total = [], [], 0.0, 0
    for nd, P, n in parts:
        off = ns.offsets_from_sizes(n)
        X = torch.from_numpy(nd.X).to(dev)
        od = torch.from_numpy(off).to(dev)
        nmax = int(n.max())
        ws = torch.empty(B.select_stencils_workspace(nd.N, nd.d, nmax), dtype=torch.uint8, device=dev)
        idx = torch.empty(int(off[-1]), dtype=torch.int32, device=dev)
        rb.select_stencils(X, od, nmax, idx=idx, workspace=ws, ctx=ctx)
        ops = ("lap", "dx", "dy") + (("dz",) if nd.d == 3 else ())
        D = rb.Domain(X, od, idx, nmax, torch.from_numpy(P).to(dev), ops)
        R = len(ops)
        csr = (torch.empty(nd.N + 1, dtype=torch.int64, device=dev), torch.empty_like(idx),
               torch.empty((R, idx.numel()), dtype=torch.float64, device=dev))
        doms.append(D)
        m = np.array([math.comb(int(p) + nd.d, nd.d) for p in P])
        nn = n.astype(np.float64)
        flop_total += float(np.sum((2.0 / 3.0) * (nn + m) ** 3 + 2.0 * R * (nn + m) ** 2 + (3 * nd.d + 1) * nn * nn))
        N_total += nd.N
        meta.append(dict(nd=nd, P=P, n=n, off=off, ws=ws, nmax=nmax, ops=ops, csr=csr))
    wsb = torch.empty(B.batched_workspace(doms), dtype=torch.uint8, device=dev)
    # the plan is tuned on a smaller batch of the same recipe (every candidate
    # plan runs the whole tuning batch), then used for the full batch
    tdoms = []
    for nd, P, n in ns.mixed_domains(a.tune_per_domain):
        off = ns.offsets_from_sizes(n)
        X = torch.from_numpy(nd.X).to(dev)
        od = torch.from_numpy(off).to(dev)
        idx = rb.select_stencils(X, od, int(n.max()), ctx=ctx)
        ops = ("lap", "dx", "dy") + (("dz",) if nd.d == 3 else ())
        tdoms.append(rb.Domain(X, od, idx, int(n.max()), torch.from_numpy(P).to(dev), ops))
    torch.cuda.synchronize()
    print(f"[bench] mixed: tuning on {sum(D.X.shape[0] for D in tdoms)} stencils", file=sys.stderr, flush=True)
    forms = [a.form] if a.no_compare else [a.form] + [f for f in ("f64", "f32_ir") if f != a.form]
    plans, tune_s = {}, {}
    for f in forms:   # per-class plans, tuned for each precision (the solvers differ)
        t = time.perf_counter()
        plans[f] = rb.autotune_batched(tdoms, precision=f, ctx=ctx)
        tune_s[f] = time.perf_counter() - t
        print(f"[bench] mixed: {f} plans {[(p['chunk'], p['waves_per_cu']) for p in plans[f]]} tuned in "
              f"{tune_s[f]:.1f} s", file=sys.stderr, flush=True)
    plan = plans[a.form]
    del tdoms
    timer = Timer(torch, ["select_stencils", "compute_weights", "assemble_csr"])

    def make_step(form):
        def step(e):
            if e:
                e[0].record(timer.stream)
            for D, mt in zip(doms, meta):
                rb.select_stencils(D.X, D.offsets, mt["nmax"], idx=D.idx, workspace=mt["ws"], ctx=ctx)
            if e:
                e[1].record(timer.stream)
            rb.compute_weights_batched(doms, precision=form, workspace=wsb, ctx=ctx)
            if e:
                e[2].record(timer.stream)
            for D, mt in zip(doms, meta):
                rp, cl, vl = mt["csr"]
                rb.assemble_csr(D.offsets, D.idx, D.w, mt["nmax"], row_ptr=rp, col=cl, vals=vl, ctx=ctx)
            if e:
                e[3].record(timer.stream)
        return step

    per = max(1, (a.err_sample if (a.no_cpu and a.err_sample) else (a.cpu_sample or 30_000)) // len(meta))
    samples = [draw_sample(mt["nd"].N, per, seed=12345 + k) for k, mt in enumerate(meta)]
    spos = [torch.from_numpy(sample_positions(mt["off"], smp)).to(dev) for mt, smp in zip(meta, samples)]
    results, snap = {}, {}
    for f in forms:
        rb.set_plan(plans[f], ctx=ctx)
        ms, wall, ph = timer.run(make_step(f), a.steps, a.warmup)
        sts = np.concatenate([D.status.cpu().numpy() for D in doms])
        results[f] = dict(form=f, ms_per_step=ms, wall_ms_per_step=wall, phases_ms=ph,
                          stencils_per_s=N_total / (ms / 1e3),
                          knn_weights_stencils_per_s=N_total / ((ph["select_stencils"] + ph["compute_weights"]) / 1e3),
                          status_counts=status_counts(sts), fallback_fraction=float(np.mean(sts == rb.ST_FALLBACK)))
        if not a.no_cpu or a.err_sample:
            snap[f] = [D.w[:, p].cpu().numpy() for D, p in zip(doms, spos)]
            if f == forms[0]:
                sidx_gpu = [D.idx[p].cpu().numpy() for D, p in zip(doms, spos)]
        print(f"[bench] mixed {f}: {ms:.3f} ms/step  phases {ph}", file=sys.stderr, flush=True)
    main = results[a.form]
    achieved = flop_total / (main["phases_ms"]["compute_weights"] / 1e3) / 1e12
    nnz_total = int(sum(mt["off"][-1] for mt in meta))
    out = base_line(a, main["stencils_per_s"], main["ms_per_step"], "f32+f64" if a.form == "f32_ir" else "f64",
                    {"workload": "mixed_2d3d_4_domains", "N": N_total, "nnz": nnz_total,
                     "domains": [dict(name=mt["nd"].meta["domain"], N=mt["nd"].N, d=mt["nd"].d) for mt in meta],
                     "n": "U[max(12, ceil(1.5 m)), 70] per node", "degree": "U{2,3,4} per node", "phs_power": 3,
                     "form": a.form, "plan": [(p["chunk"], p["waves_per_cu"]) for p in plan],
                     "class_sizes": rb.batched_class_sizes(), "autotune_s": tune_s,
                     "tune_per_domain": a.tune_per_domain,
                     "step": "select_stencils x4 + compute_weights_batched + assemble_csr x4"})
    out["roofline"] = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                       "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                       "kernel": "k_bclass, k_bclass_pair, k_bclass_quad: one persistent launch per size class "
                                 "(refined pass + FP64 fallback pass)" if a.form == "f32_ir"
                       else "k_bclass, k_bclass_quad: one persistent launch per size class", "flop_per_stencil": flop_total / N_total, "stencils_per_launch": N_total}
    out["forms"] = results
    if "f64" in results and "f32_ir" in results:
        out["mixed_vs_f64"] = (results["f32_ir"]["knn_weights_stencils_per_s"] /
                               results["f64"]["knn_weights_stencils_per_s"])
    if not a.no_cpu:
        tot_n, tot_t, err, cores = 0, 0.0, {}, 1
        for k, mt in enumerate(meta):
            sample = samples[k]
            base, soff, sidx, Wo = cpu_oracle(mt["nd"].X, mt["n"], mt["P"].astype(np.int64), mt["ops"], sample)
            tot_n += sample.size
            tot_t += sample.size / base["value"]
            cores = max(cores, base["cores"])
            s = {f: (snap[f][k], None) for f in snap}
            e = sample_errors(s, sample, soff, sidx, Wo, mt["ops"], mt["nd"].h[sample])
            for f, v in e.items():
                err.setdefault(f, []).append(v["scaled_max_err"])
        out["cpu_baseline"] = {"value": tot_n / tot_t, "unit": "stencils/s", "cores": cores, "kind": "oracle",
                               "sample": f"{tot_n} seeded random nodes over the 4 domains "
                                         f"(kNN against all nodes + weights), BLAS limited to one thread"}
        out["error"] = {f: {"scaled_max_err": max(v), "tolerance": 1e-10 if f == "f64" else 1e-9}
                        for f, v in err.items()}
    elif a.err_sample:
        from oracle import rbffd as orbf
        err = {}
        for k, mt in enumerate(meta):
            sample = samples[k]
            soff = ns.offsets_from_sizes(mt["n"][sample])
            Wo, _ = orbf.weights(mt["nd"].X, soff, sidx_gpu[k], mt["P"][sample].astype(np.int64), mt["ops"])
            e = sample_errors({f: (snap[f][k], None) for f in snap}, sample, soff, None, Wo, mt["ops"],
                              mt["nd"].h[sample])
            for f, v in e.items():
                err.setdefault(f, []).append(v["scaled_max_err"])
        out["error"] = {f: {"scaled_max_err": max(v), "tolerance": 1e-10 if f == "f64" else 1e-9,
                            "sample": int(sum(x.size for x in samples))} for f, v in err.items()}
        out["error"]["note"] = "oracle weights of the GPU's stencils"
    return out


# ---------------------------------------------------------------- learned surrogate
def bench_learned(a, torch, rb, B):
    import nodesets as ns
    from paper_1912_13282_amd import surrogate as S
    dev = torch.device("cuda:0")
    t = time.perf_counter()
    data = S.build_training_set(S.training_node_sets(a.train_sets), device=dev)
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t
    S_n = data.feat.shape[0]
    st = S.TrainState.init(22, device=dev)
    batch = 8192
    torch.cuda.synchronize()
    t = time.perf_counter()
    hist = S.train(st, data, epochs=a.train_epochs, batch=batch, lr=2e-3, seed=4)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t
    print(f"[bench] learned: {S_n} training stencils prepared in {prep_s:.1f} s; {st.step} Adam steps "
          f"in {train_s:.1f} s, loss {hist[0]:.3e} -> {hist[-1]:.3e}", file=sys.stderr, flush=True)
    del data

    # quality on the 2,007-node disk (seed 1001)
    from oracle import poisson as opoi
    q = ns.disk(ns.DISK_H, 1001)
    Xq = torch.from_numpy(q.X).to(dev)
    oq = torch.arange(0, (q.N + 1) * 15, 15, dtype=torch.int64, device=dev)
    iq = rb.select_stencils(Xq, oq, 15)
    wpq, _ = rb.compute_weights(Xq, oq, iq, 15, 2, ("lap",), precision="f64")
    wtq, stq = S.surrogate_laplacian(Xq, oq, iq, st.params)
    wzq, _ = S.surrogate_laplacian(Xq, oq, iq, torch.zeros_like(st.params), corr_tol=float("inf"))  # ablation
    iqn = iq.cpu().numpy()
    quality = {}
    for nm, wv in (("plain", wpq[0]), ("trained", wtq), ("zero_network", wzq)):
        wn = wv.cpu().numpy()
        approx = (wn * opoi.u0(q.X)[iqn]).reshape(-1, 15).sum(1)
        quality[nm] = {"poisson_max_err": opoi.solve_dirichlet(q.X, q.is_boundary, oq.cpu().numpy(), iqn, wn)[1],
                       "e_h": float(np.abs(approx - opoi.lap_u0(q.X))[~q.is_boundary].max())}
    quality["accepted_fraction"] = float((stq.cpu().numpy() == rb.ST_SURROGATE).mean())
    # the acceptance gate on the projection's correction, max|w - y| <= corr_tol max|w|: tighter
    # gates send more stencils to the plain solve and bring the Poisson error towards the plain one
    quality["gate_sweep"] = []
    for ct in (0.25, 0.1, 0.05, 0.02):
        wg, sg = S.surrogate_laplacian(Xq, oq, iq, st.params, corr_tol=ct)
        quality["gate_sweep"].append({
            "corr_tol": ct, "accepted_fraction": float((sg.cpu().numpy() == rb.ST_SURROGATE).mean()),
            "poisson_max_err": opoi.solve_dirichlet(q.X, q.is_boundary, oq.cpu().numpy(), iqn, wg.cpu().numpy())[1]})

    # throughput on a 1.7M-node disk
    nd = ns.disk(ns.DISK_H / 30.0, 1001)
    N = nd.N
    X = torch.from_numpy(nd.X).to(dev)
    off = torch.arange(0, (N + 1) * 15, 15, dtype=torch.int64, device=dev)
    idx = torch.empty(N * 15, dtype=torch.int32, device=dev)
    ws = torch.empty(B.select_stencils_workspace(N, 2, 15), dtype=torch.uint8, device=dev)
    w = torch.empty((1, N * 15), dtype=torch.float64, device=dev)
    status = torch.empty(N, dtype=torch.int8, device=dev)
    ctx = rb.context(dev)
    B.surrogate_load(st.params, ctx=ctx)
    timer = Timer(torch, ["select_stencils", "compute_weights"])

    def make_step(form):
        def step(e):
            if e:
                e[0].record(timer.stream)
            rb.select_stencils(X, off, 15, idx=idx, workspace=ws, ctx=ctx)
            if e:
                e[1].record(timer.stream)
            if form == "surrogate":
                B.surrogate_weights(X, off, idx, 15, w=w[0], status=status, ctx=ctx)
            else:
                rb.compute_weights(X, off, idx, 15, 2, ("lap",), precision=form, w=w, status=status, ctx=ctx)
            if e:
                e[2].record(timer.stream)
        return step

    results = {}
    forms = ["surrogate"] if a.no_compare else ["surrogate", "f64", "f32_ir"]
    wsnap = {}
    for f in forms:
        ms, wall, ph = timer.run(make_step(f), a.steps, a.warmup)
        stn = status.cpu().numpy()
        results[f] = dict(form=f, ms_per_step=ms, wall_ms_per_step=wall, phases_ms=ph,
                          stencils_per_s=N / (ms / 1e3), status_counts=status_counts(stn))
        wsnap[f] = w[0].cpu().numpy()
        print(f"[bench] learned {f}: {ms:.3f} ms/step  phases {ph}", file=sys.stderr, flush=True)
    main = results["surrogate"]
    if "f64" in wsnap:
        dv = (np.abs(wsnap["surrogate"] - wsnap["f64"]).reshape(-1, 15).max(1) /
              np.abs(wsnap["f64"]).reshape(-1, 15).max(1))
        quality["deviation_from_plain"] = {"median": float(np.median(dv)), "p99": float(np.quantile(dv, 0.99)),
                                           "max": float(dv.max())}
    t_w = main["phases_ms"]["compute_weights"] / 1e3
    achieved = SURROGATE_FLOPS * N / t_w / 1e12
    out = base_line(a, main["stencils_per_s"], main["ms_per_step"], "bf16+f32+f64",
                    {"workload": "learned_laplacian_disk_2d", "N": N, "n": 15, "degree": 2, "m": 6, "ops": ["lap"],
                     "network": "30-128-128-128-15 GELU", "training_stencils": S_n, "train_epochs": a.train_epochs,
                     "batch": batch, "adam_steps": st.step, "train_s": train_s,
                     "train_samples_per_s": st.step * batch / train_s, "loss_first_last": [hist[0], hist[-1]],
                     "step": "select_stencils + surrogate_weights (projection + plain-solve fallback)"})
    out["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                       "frac": achieved / PEAK_BF16_TFLOPS, "traffic": None,
                       "kernel": "k_surrogate + k_weights_f64<24> (fallback pass)",
                       "flop_per_stencil": SURROGATE_FLOPS, "stencils_per_launch": N,
                       "hbm_GBs_algorithmic": SURROGATE_BYTES * N / t_w / 1e9}
    out["forms"] = results
    out["quality"] = quality
    if "f64" in results:
        out["learned_vs_f64"] = main["stencils_per_s"] / results["f64"]["stencils_per_s"]
    if not a.no_cpu:
        base, soff, sidx, Wo = cpu_oracle(nd.X, 15, 2, ("lap",), draw_sample(N, a.cpu_sample or 30_000))
        out["cpu_baseline"] = base
    return out


# ---------------------------------------------------------------- GWLS engine (Sec. 2.2.1)
def wls_flops(n, m, R, d):
    """Algorithmic FLOPs of one stencil's GWLS weights by Householder QR: the
    factorisation of the n x m matrix W B (2 n m^2 - 2 m^3 / 3), per operator the
    substitution with R^T (m^2) and the reflections applied to [z; 0] (4 n m - 2 m^2),
    and the basis and weight-function values (about n (m + 2 d + 10))."""
    return 2.0 * n * m * m - 2.0 * m ** 3 / 3.0 + R * (m * m + 4.0 * n * m - 2.0 * m * m) + n * (m + 2 * d + 10)


def bench_wls(a, torch, rb, B):
    import nodesets as ns
    dev = torch.device("cuda:0")
    wl = ns.workload("cube_sphere3d")
    nd = wl["nodes"][0]
    n, P, ops = wl["n"], wl["P"], wl["ops"]
    N, d, R = nd.N, nd.d, len(ops)
    m = math.comb(P + d, d)
    sigma = 1.0
    off_h = ns.offsets_from_sizes(np.full(N, n, dtype=np.int64))
    nnz = int(off_h[-1])
    X = torch.from_numpy(nd.X).to(dev)
    offsets = torch.from_numpy(off_h).to(dev)
    idx = torch.empty(nnz, dtype=torch.int32, device=dev)
    ws = torch.empty(B.select_stencils_workspace(N, d, n), dtype=torch.uint8, device=dev)
    w = torch.empty((R, nnz), dtype=torch.float64, device=dev)
    status = torch.empty(N, dtype=torch.int8, device=dev)
    row_ptr = torch.empty(N + 1, dtype=torch.int64, device=dev)
    col = torch.empty(nnz, dtype=torch.int32, device=dev)
    vals = torch.empty((R, nnz), dtype=torch.float64, device=dev)
    ctx = rb.context(dev)
    timer = Timer(torch, ["select_stencils", "compute_weights_wls", "assemble_csr"])

    def step(e):
        if e:
            e[0].record(timer.stream)
        rb.select_stencils(X, offsets, n, idx=idx, workspace=ws, ctx=ctx)
        if e:
            e[1].record(timer.stream)
        rb.compute_weights_wls(X, offsets, idx, n, P, ops, weight="gaussian", sigma=sigma, w=w, status=status,
                               ctx=ctx)
        if e:
            e[2].record(timer.stream)
        rb.assemble_csr(offsets, idx, w, n, row_ptr=row_ptr, col=col, vals=vals, ctx=ctx)
        if e:
            e[3].record(timer.stream)

    ms, wall, ph = timer.run(step, a.steps, a.warmup)
    st = status.cpu().numpy()
    print(f"[bench] wls: {ms:.3f} ms/step  phases {ph}", file=sys.stderr, flush=True)
    flop = wls_flops(n, m, R, d)
    achieved = flop * N / (ph["compute_weights_wls"] / 1e3) / 1e12
    res = base_line(a, N / (ms / 1e3), ms, "f64",
                    {"workload": "wls_cube_minus_sphere_3d", "N": N, "nnz": nnz, "n": n, "degree": P, "m": m,
                     "ops": list(ops), "weight": "gaussian", "sigma": sigma,
                     "step": "select_stencils + compute_weights_wls + assemble_csr"})
    res["metric"] = "GWLS stencils/s (kNN + weights + CSR)"
    res["roofline"] = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                       "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None, "kernel": "k_wls<20>",
                       "flop_per_stencil": flop, "stencils_per_launch": N}
    res["phases_ms"] = ph
    res["wall_ms_per_step"] = wall
    res["status_counts"] = status_counts(st)
    if not a.no_cpu:
        from threadpoolctl import threadpool_limits

        from oracle import knn as oknn
        from oracle import wls as owls
        sample = draw_sample(N, a.cpu_sample or 60_000)
        snap = w[:, torch.from_numpy(sample_positions(off_h, sample)).to(dev)].cpu().numpy()
        with threadpool_limits(limits=1):
            t = time.perf_counter()
            c0 = time.process_time()
            soff, sidx = oknn.knn_exact(nd.X, n, nodes=sample)
            Wo = np.concatenate([owls.stencil_weights(nd.X[sidx[soff[i]:soff[i + 1]]], P, ops, owls.GAUSSIAN, sigma)
                                 for i in range(sample.size)], axis=1)
            dt = time.perf_counter() - t
            cpu_s = time.process_time() - c0
        res["cpu_baseline"] = {"value": sample.size / dt, "unit": "stencils/s", "cores": max(1, int(round(cpu_s / dt))),
                               "kind": "oracle",
                               "sample": f"{sample.size} seeded random nodes of the same workload (kNN against all "
                                         f"{N} nodes + GWLS weights by pseudo-inverse), {dt:.1f} s wall, "
                                         f"{cpu_s:.1f} s CPU, BLAS limited to one thread"}
        res["error"] = {"scaled_max_err": scaled_err(snap, Wo, ops, np.repeat(nd.h[sample], n)),
                        "tolerance": 1e-10, "sample": int(sample.size)}
    return res


# ---------------------------------------------------------------- explicit heat step
def explicit_bytes(n_int, n_dir, n_neu, n, d, N):
    """Algorithmic HBM bytes of one explicit step: per node its kind, row offset,
    own value and result (the field is read once); interior rows the stencil
    indices, Laplacian weights and source; Dirichlet rows g; Neumann rows the
    indices, d gradient weight rows, the normal and g."""
    return (N * (1 + 8 + 8 + 8) + n_int * (12.0 * n + 8) + n_dir * 8 +
            n_neu * (4.0 * n + 8.0 * d * n + 8 * d + 8))


def apply_bytes(N, n, R):
    """Algorithmic HBM bytes of one application of R operators: row offsets,
    indices, R weight rows, the field once and R outputs."""
    return N * (8 + 4.0 * n + 8.0 * R * n + 8 + 8.0 * R)


def bench_explicit(a, torch, rb, B):
    import nodesets as ns
    dev = torch.device("cuda:0")
    wl = ns.workload("cube_sphere3d")
    nd = wl["nodes"][0]
    n, P, ops = wl["n"], wl["P"], wl["ops"]
    N, d, R = nd.N, nd.d, len(wl["ops"])
    c = np.array([0.5, 0.5, 0.5])
    r = np.linalg.norm(nd.X - c, axis=1)
    sphere = nd.is_boundary & (r < 0.3 + 1e-9)
    kind = np.where(nd.is_boundary, rb.NODE_DIRICHLET, rb.NODE_INTERIOR).astype(np.uint8)
    kind[sphere] = rb.NODE_NEUMANN
    normals = np.zeros((N, 3))
    normals[sphere] = (c - nd.X[sphere]) / r[sphere, None]
    g = np.where(kind == rb.NODE_DIRICHLET, nd.X[:, 0], 0.0)
    counts = [int((kind == k).sum()) for k in (rb.NODE_INTERIOR, rb.NODE_DIRICHLET, rb.NODE_NEUMANN)]
    X = torch.from_numpy(nd.X).to(dev)
    off_h = ns.offsets_from_sizes(np.full(N, n, dtype=np.int64))
    off = torch.from_numpy(off_h).to(dev)
    ctx = rb.context(dev)
    idx = rb.select_stencils(X, off, n, ctx=ctx)
    w, st = rb.compute_weights(X, off, idx, n, P, ops, precision="f64", ctx=ctx)
    kt, nt, gt = (torch.from_numpy(v).to(dev) for v in (kind, normals, g))
    s = torch.full((N,), 5.0, dtype=torch.float64, device=dev)
    u = torch.where(kt == rb.NODE_DIRICHLET, gt, torch.zeros_like(gt))
    v = torch.empty_like(u)
    out = torch.empty((R, N), dtype=torch.float64, device=dev)
    h = ns.CUBE_SPHERE_H
    dt = 0.02 * h * h
    timer = Timer(torch, ["explicit_step", "apply_operators"])
    # the first step from u = 0 (the field stays bounded over the timed steps)
    fields = [u, v]

    def step(e):
        if e:
            e[0].record(timer.stream)
        rb.explicit_step(off, idx, n, w[0], kt, fields[0], dt, w_grad=w[1:], normals=nt, g=gt, s=s, out=fields[1],
                         ctx=ctx)
        if e:
            e[1].record(timer.stream)
        rb.apply_operators(off, idx, w, n, fields[1], out=out, ctx=ctx)
        if e:
            e[2].record(timer.stream)
        fields.reverse()

    ms, wall, ph = timer.run(step, a.steps, a.warmup)
    print(f"[bench] explicit: {ms:.4f} ms/step  phases {ph}", file=sys.stderr, flush=True)
    eb = explicit_bytes(*counts, n, d, N)
    ab = apply_bytes(N, n, R)
    gbs_e = eb / (ph["explicit_step"] / 1e3) / 1e9
    gbs_a = ab / (ph["apply_operators"] / 1e3) / 1e9
    res = base_line(a, N / (ms / 1e3), ms, "f64",
                    {"workload": "explicit_heat_cube_minus_sphere_3d", "N": N, "nnz": N * n, "n": n, "degree": P,
                     "ops": list(ops), "interior_dirichlet_neumann": counts, "dt": dt,
                     "step": "explicit_step (du/dt = lap u + 5; faces u = x, sphere zero flux) + "
                             "apply_operators (lap, dx, dy, dz of the new field)"})
    res["metric"] = "explicit Euler node updates/s (one step + evaluation of four operators)"
    res["unit"] = "nodes/s"
    res["roofline"] = {"bound": "hbm", "achieved": gbs_a, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                       "frac": gbs_a / PEAK_HBM_GBS, "traffic": recorded_traffic("explicit"),
                       "kernel": "k_apply<8,5,4>", "bytes_per_node": ab / N, "nodes_per_launch": N}
    res["phases_roofline"] = {"explicit_step": {"bound": "hbm", "kernel": "k_explicit<8,5>", "bytes": eb,
                                                "achieved_GBs": gbs_e, "frac": gbs_e / PEAK_HBM_GBS},
                              "apply_operators": {"bound": "hbm", "kernel": "k_apply<8,5,4>", "bytes": ab,
                                                  "achieved_GBs": gbs_a, "frac": gbs_a / PEAK_HBM_GBS}}
    res["phases_ms"] = ph
    res["wall_ms_per_step"] = wall
    finite = bool(torch.isfinite(fields[0]).all().item())
    res["field_finite"] = finite
    if a.calib_copy:
        calib_copy(torch, dev)
    if not a.no_cpu:
        res["cpu_baseline"] = cpu_explicit(nd, kind, normals, g, off_h, idx.cpu().numpy(), w.cpu().numpy(),
                                           fields[0].cpu().numpy(), dt, N)
    return res


def cpu_explicit(nd, kind, normals, g, off, idx, W, u, dt, sample):
    """The oracle's explicit step and operator application on the first `sample`
    rows (about 5 us per row: the whole node set fits the time budget), one thread."""
    from threadpoolctl import threadpool_limits

    from oracle import explicit as oexp
    S = min(sample, nd.N)
    so, si = off[:S + 1], idx[:off[S]]
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        c0 = time.process_time()
        oexp.explicit_step(so, si, W[0][:off[S]], W[1:, :off[S]], kind[:S], normals[:S], u, dt, g=g[:S],
                           s=np.full(S, 5.0))
        oexp.apply_operators(so, si, W[:, :off[S]], u)
        dtw = time.perf_counter() - t
        cpu_s = time.process_time() - c0
    return {"value": S / dtw, "unit": "nodes/s", "cores": max(1, int(round(cpu_s / dtw))), "kind": "oracle",
            "sample": f"{S} of {nd.N} nodes of the same workload (one explicit step + four operators), "
                      f"{dtw:.1f} s wall, {cpu_s:.1f} s CPU, BLAS limited to one thread"}


# ---------------------------------------------------------------- implicit Poisson (Sec. 5)
POISSON_CASES = {
    # name: (d, n, degree, h) -- the annulus B(0,1) minus B(0,1/2); about 1M nodes each
    "poisson3d": (3, 35, 2, 0.0154),
    "poisson2d": (2, 9, 2, 0.00154),
}


def bicgstab_bytes_per_row(n, precond="jacobi"):
    """Algorithmic HBM bytes per row of one BiCGStab iteration: two row products
    (row offset, n indices and values, the gathered vector once, the inverse
    diagonal, one dot operand, the result) and the three vector passes
    (p: 3 reads + 1 write, s: 2 + 1, x and r: 5 + 2).  Block-Jacobi adds to the
    p and s passes the block product of each row: 64 float16 entries of the
    inverse, its float32 scale, the permutation entry and the output."""
    b = 2 * (8 + 12.0 * n + 8 + 8 + 8 + 8) + 8 * (4 + 3 + 7)
    if precond == "block_jacobi":
        b += 2 * (64 * 2 + 4 + 4 + 8)
    return b


def bench_poisson(a, torch, rb, B):
    import nodesets as ns
    from oracle import poisson as opoi
    dev = torch.device("cuda:0")
    d, n, P, h = POISSON_CASES[a.workload]
    t = time.perf_counter()
    nd = ns.annulus(h, 1006, d=d)
    N = nd.N
    print(f"[bench] {a.workload}: {N} nodes generated in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    X = torch.from_numpy(nd.X).to(dev)
    off = torch.from_numpy(ns.offsets_from_sizes(np.full(N, n, dtype=np.int64))).to(dev)
    nnz = N * n
    ctx = rb.context(dev)
    idx = torch.empty(nnz, dtype=torch.int32, device=dev)
    ws = torch.empty(B.select_stencils_workspace(N, d, n), dtype=torch.uint8, device=dev)
    w = torch.empty((1, nnz), dtype=torch.float64, device=dev)
    status = torch.empty(N, dtype=torch.int8, device=dev)
    kind = torch.from_numpy(np.where(nd.is_boundary, rb.NODE_DIRICHLET, rb.NODE_INTERIOR).astype(np.uint8)).to(dev)
    u0 = opoi.u0(nd.X)
    f = torch.from_numpy(opoi.lap_u0(nd.X)).to(dev)
    g = torch.from_numpy(u0).to(dev)
    vals = torch.empty(nnz, dtype=torch.float64, device=dev)
    rhs = torch.empty(N, dtype=torch.float64, device=dev)
    x = torch.empty(N, dtype=torch.float64, device=dev)
    sws = torch.empty(rb.bicgstab_workspace(N, nnz, "block_jacobi"), dtype=torch.uint8, device=dev)  # the larger form
    tol = 1e-10
    # auto: block-Jacobi where its block products are small against the row
    # products (3D, 35 entries per row); with 9 entries per row (2D) the block
    # products nearly double an iteration's bytes and the matrix no longer stays
    # in the last-level cache, for a smaller cut in iterations
    if a.precond == "auto":
        a.precond = "block_jacobi" if d == 3 else "jacobi"
    bj = a.precond == "block_jacobi"
    pc = torch.empty(rb.block_jacobi_size(N, d), dtype=torch.uint8, device=dev)
    timer = Timer(torch, ["select_stencils", "compute_weights", "assemble_implicit", "precondition", "bicgstab"])
    infos = []

    def solve(precond):
        x.zero_()
        return rb.bicgstab(off, idx, vals, n, rhs, x=x, tol=tol, max_iter=100000, precond=precond,
                           workspace=sws, ctx=ctx, pc=pc if precond == "block_jacobi" else None)[1]

    def step(e):
        if e:
            e[0].record(timer.stream)
        rb.select_stencils(X, off, n, idx=idx, workspace=ws, ctx=ctx)
        if e:
            e[1].record(timer.stream)
        rb.compute_weights(X, off, idx, n, P, ("lap",), precision="f64", w=w, status=status, ctx=ctx)
        if e:
            e[2].record(timer.stream)
        rb.assemble_implicit(off, idx, w[0], kind, f=f, g=g, d=d, vals=vals, rhs=rhs, ctx=ctx)
        if e:
            e[3].record(timer.stream)
        if bj:
            rb.block_jacobi(X, off, idx, vals, pc=pc, ctx=ctx)
        if e:
            e[4].record(timer.stream)
        infos.append(solve(a.precond))
        if e:
            e[5].record(timer.stream)

    ms, wall, ph = timer.run(step, a.steps, a.warmup)
    info = infos[-1]
    err = float(np.abs(x.cpu().numpy() - u0).max())
    print(f"[bench] {a.workload}: {ms:.2f} ms/step  phases {ph}  solve {info}  max error {err:.3e}",
          file=sys.stderr, flush=True)
    it = max(1, info["iterations"])
    per_row = bicgstab_bytes_per_row(n, a.precond)
    gbs = per_row * N * it / (ph["bicgstab"] / 1e3) / 1e9
    solver = {"block_jacobi": "BiCGStab, block-Jacobi (64-node cell blocks, float16 inverses)",
              "jacobi": "BiCGStab, Jacobi row scaling", "none": "BiCGStab, unpreconditioned"}[a.precond]
    res = base_line(a, N / (ms / 1e3), ms, "f64",
                    {"workload": f"poisson_annulus_{d}d", "N": N, "nnz": nnz, "n": n, "degree": P, "ops": ["lap"],
                     "solver": solver, "tol": tol,
                     "step": "select_stencils + compute_weights + assemble_implicit + precondition + bicgstab"})
    res["metric"] = "Poisson nodes solved/s (stencils + weights + assembly + BiCGStab)"
    res["unit"] = "nodes/s"
    vp, vs = ("k_bj_vec<P>", "k_bj_vec<S>") if bj else ("k_vec<P>", "k_vec<S>")
    res["roofline"] = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                       "frac": gbs / PEAK_HBM_GBS, "traffic": recorded_traffic(a.workload),
                       "kernel": f"BiCGStab iteration ({vp}, k_spmv<V>, {vs}, k_spmv<T>, k_vec<X>; "
                                 f"row products k_spmv<8,{(n + 7) // 8}>)",
                       "bytes_per_row_per_iteration": per_row, "rows": N, "iterations": it}
    if not a.no_compare:
        # the other preconditioner on the same system, one untimed-by-the-step solve
        other = "jacobi" if bj else "block_jacobi"
        if other == "block_jacobi":
            rb.block_jacobi(X, off, idx, vals, pc=pc, ctx=ctx)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(timer.stream)
        oi = solve(other)
        t1.record(timer.stream)
        torch.cuda.synchronize()
        res["compare_precond"] = {"precond": other, "iterations": oi["iterations"], "status": oi["status"],
                                  "bicgstab_ms": t0.elapsed_time(t1)}
        print(f"[bench] {a.workload}: with {other}: {res['compare_precond']}", file=sys.stderr, flush=True)
    res["phases_ms"] = ph
    res["wall_ms_per_step"] = wall
    res["solve"] = info
    res["max_error_vs_u0"] = err
    if a.calib_copy:
        calib_copy(torch, dev)
    if not a.no_cpu:
        res["cpu_baseline"] = cpu_poisson(d, n, P)
    return res


def cpu_poisson(d, n, P):
    """The oracle pipeline (exact kNN, weights by LAPACK per stencil, assembly,
    sparse direct solve) on a smaller annulus of the same kind, one BLAS thread."""
    from threadpoolctl import threadpool_limits

    import nodesets as ns
    from oracle import implicit as oimp
    from oracle import knn as oknn
    from oracle import poisson as opoi
    from oracle import rbffd as orbf
    h = 0.06 if d == 3 else 0.012
    nd = ns.annulus(h, 1006, d=d)
    N = nd.N
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        c0 = time.process_time()
        off, idx = oknn.knn_exact(nd.X, n)
        W, _ = orbf.weights(nd.X, off, idx, P, ("lap",))
        kind = np.where(nd.is_boundary, oimp.DIRICHLET, oimp.INTERIOR)
        vals, rhs = oimp.assemble(off, idx, W[0], None, kind, None, f=opoi.lap_u0(nd.X), g=opoi.u0(nd.X))
        oimp.solve(off, idx, vals, rhs)
        dt = time.perf_counter() - t
        cpu_s = time.process_time() - c0
    return {"value": N / dt, "unit": "nodes/s", "cores": max(1, int(round(cpu_s / dt))), "kind": "oracle",
            "sample": f"the same problem on a coarser annulus (h = {h}, {N} nodes): kNN + weights + assembly + "
                      f"sparse direct solve, {dt:.1f} s wall, {cpu_s:.1f} s CPU, BLAS limited to one thread"}


def bench_counters(a, torch, rb, B):
    """One launch of each hot kernel at its workload's shape (see the module
    docstring), nothing timed: the command profiled by the counter passes."""
    import nodesets as ns
    dev = torch.device("cuda:0")
    ctx = rb.context(dev)
    ran = []

    def uniform(nd, n, P, ops, forms):
        off = torch.from_numpy(ns.offsets_from_sizes(np.full(nd.N, n, dtype=np.int64))).to(dev)
        X = torch.from_numpy(nd.X).to(dev)
        idx = rb.select_stencils(X, off, n, ctx=ctx)
        for f in forms:
            w, _ = rb.compute_weights(X, off, idx, n, P, ops, precision=f, ctx=ctx)
        rb.assemble_csr(off, idx, w, n, ctx=ctx)
        torch.cuda.synchronize()
        ran.append(dict(N=nd.N, n=n, degree=P, forms=list(forms)))
        print(f"[bench] counters: {ran[-1]}", file=sys.stderr, flush=True)
        return off, idx, w

    wl = ns.workload("cube_sphere3d")
    nd = wl["nodes"][0]
    off, idx, w = uniform(nd, wl["n"], wl["P"], wl["ops"], ("f64", "f32_ir"))
    # the explicit workload's kernels on the same stencils: the four operators
    # applied to a field, and one explicit step with Dirichlet rows only
    u = torch.from_numpy(np.sin(nd.X[:, 0]) * nd.X[:, 1]).to(dev)
    rb.apply_operators(off, idx, w, wl["n"], u, ctx=ctx)
    kt = torch.from_numpy(np.where(nd.is_boundary, rb.NODE_DIRICHLET, rb.NODE_INTERIOR).astype(np.uint8)).to(dev)
    rb.explicit_step(off, idx, wl["n"], w[0], kt, u, 0.02 * ns.CUBE_SPHERE_H ** 2, g=u, ctx=ctx)
    torch.cuda.synchronize()
    ran.append(dict(explicit_N=nd.N))
    print(f"[bench] counters: {ran[-1]}", file=sys.stderr, flush=True)
    del off, idx, w, u, kt
    # the 3D Poisson system of Sec. 5: twenty BiCGStab iterations with each preconditioner
    from oracle import poisson as opoi
    d3, n3, P3, h3 = POISSON_CASES["poisson3d"]
    nd = ns.annulus(h3, 1006, d=d3)
    X = torch.from_numpy(nd.X).to(dev)
    off = torch.from_numpy(ns.offsets_from_sizes(np.full(nd.N, n3, dtype=np.int64))).to(dev)
    idx = rb.select_stencils(X, off, n3, ctx=ctx)
    w, _ = rb.compute_weights(X, off, idx, n3, P3, ("lap",), precision="f64", ctx=ctx)
    kind = torch.from_numpy(np.where(nd.is_boundary, rb.NODE_DIRICHLET, rb.NODE_INTERIOR).astype(np.uint8)).to(dev)
    vals, rhs = rb.assemble_implicit(off, idx, w[0], kind, f=torch.from_numpy(opoi.lap_u0(nd.X)).to(dev),
                                     g=torch.from_numpy(opoi.u0(nd.X)).to(dev), d=d3, ctx=ctx)
    pc = rb.block_jacobi(X, off, idx, vals, ctx=ctx)
    for pre in ("jacobi", "block_jacobi"):
        rb.bicgstab(off, idx, vals, n3, rhs, tol=1e-30, max_iter=20, precond=pre, ctx=ctx, pc=pc)
    torch.cuda.synchronize()
    ran.append(dict(poisson3d_N=nd.N, iterations=20, preconds=["jacobi", "block_jacobi"]))
    print(f"[bench] counters: {ran[-1]}", file=sys.stderr, flush=True)
    del X, off, idx, w, kind, vals, rhs, pc
    wl = ns.workload("large3d", h=1.0 / 100)
    uniform(wl["nodes"][0], wl["n"], wl["P"], wl["ops"], ("f64", "f32_ir"))
    doms = []
    for nd, P, n in ns.mixed_domains(200_000):
        off = torch.from_numpy(ns.offsets_from_sizes(n)).to(dev)
        X = torch.from_numpy(nd.X).to(dev)
        idx = rb.select_stencils(X, off, int(n.max()), ctx=ctx)
        doms.append(rb.Domain(X, off, idx, int(n.max()), torch.from_numpy(P).to(dev),
                              ("lap", "dx", "dy") + (("dz",) if nd.d == 3 else ())))
    for f in ("f64", "f32_ir"):
        rb.compute_weights_batched(doms, precision=f, ctx=ctx)
    torch.cuda.synchronize()
    ran.append(dict(mixed_stencils=int(sum(D.X.shape[0] for D in doms)), forms=["batched f64", "batched f32_ir"]))
    print(f"[bench] counters: {ran[-1]}", file=sys.stderr, flush=True)
    del doms
    # the surrogate: a seeded network (its operation counts do not depend on the values)
    nd = ns.disk(ns.DISK_H / 30.0, 1001)
    off = torch.from_numpy(ns.offsets_from_sizes(np.full(nd.N, 15, dtype=np.int64))).to(dev)
    X = torch.from_numpy(nd.X).to(dev)
    idx = rb.select_stencils(X, off, 15, ctx=ctx)
    B.surrogate_load(B.mlp_flatten(ns.surrogate_init(4)).to(dev), ctx=ctx)
    B.surrogate_weights(X, off, idx, 15, ctx=ctx)
    torch.cuda.synchronize()
    ran.append(dict(surrogate_N=nd.N))
    calib_copy(torch, dev)
    return {"workload": "counters", "ran": ran}


def leg_summary(o):
    keep = ("value", "unit", "ms_per_step", "dtype", "config", "roofline", "phases_roofline", "mixed_vs_f64", "error")
    r = {k: o[k] for k in keep if k in o}
    r["forms"] = {f: {k: v[k] for k in ("ms_per_step", "phases_ms", "stencils_per_s", "knn_weights_stencils_per_s",
                                          "status_counts", "fallback_fraction")}
                  for f, v in o["forms"].items()}
    return r


def legs(a, torch, rb, B):
    """Compact runs of the other three throughput workloads, reported beside the
    main line: the 16.3M-node large-3D set (plain FP64 vs FP32+refine vs the
    batched persistent form, with CSR), the 8.1M-stencil mixed 2D/3D batch
    (per-class plans tuned per precision), one warm-up and one timed step per
    form, weights checked against the oracle on a seeded sample; and the learned
    Laplacian (training on the GPU, then the surrogate against FP64 and FP32 +
    refinement on a 1.7M-node disk, three timed steps)."""
    import copy
    out = {}
    la = copy.copy(a)
    la.steps, la.warmup, la.no_cpu, la.err_sample, la.no_compare = 1, 1, True, 2000, False
    la.batched_forms, la.calib_copy = True, False
    t = time.perf_counter()
    out["large3d"] = leg_summary(bench_uniform(la, torch, rb, B, "large3d"))
    out["large3d"]["leg_wall_s"] = time.perf_counter() - t
    torch.cuda.empty_cache()
    lm = copy.copy(la)
    lm.batched_forms = False
    t = time.perf_counter()
    out["mixed"] = leg_summary(bench_mixed(lm, torch, rb, B))
    out["mixed"]["leg_wall_s"] = time.perf_counter() - t
    torch.cuda.empty_cache()
    ll = copy.copy(la)
    ll.steps, ll.warmup = 3, 1
    t = time.perf_counter()
    o = bench_learned(ll, torch, rb, B)
    out["learned"] = {k: o[k] for k in ("value", "unit", "ms_per_step", "dtype", "config", "roofline", "quality",
                                        "learned_vs_f64") if k in o}
    out["learned"]["forms"] = {f: {k: v[k] for k in ("ms_per_step", "phases_ms", "stencils_per_s", "status_counts")}
                               for f, v in o["forms"].items()}
    out["learned"]["leg_wall_s"] = time.perf_counter() - t
    torch.cuda.empty_cache()
    return out


def main():
    a = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for {max(a.gpus, world)}); "
              "the path shards by node ranges with a halo exchange, which this build does not run.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1912_13282_amd as rb
    from paper_1912_13282_amd import _binding as B

    torch.cuda.set_device(torch.device("cuda:0"))
    if a.workload in ("cube_sphere3d", "large3d"):
        out = bench_uniform(a, torch, rb, B, a.workload)
        if a.workload == "cube_sphere3d" and not a.no_legs:
            out["legs"] = legs(a, torch, rb, B)
    elif a.workload == "mixed":
        out = bench_mixed(a, torch, rb, B)
    elif a.workload == "explicit":
        out = bench_explicit(a, torch, rb, B)
    elif a.workload == "wls":
        out = bench_wls(a, torch, rb, B)
    elif a.workload == "counters":
        out = bench_counters(a, torch, rb, B)
    elif a.workload in POISSON_CASES:
        out = bench_poisson(a, torch, rb, B)
    else:
        out = bench_learned(a, torch, rb, B)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
