"""Benchmark of the RBF-FD stencil hot path on one MI355X.

One step = rbf_select_stencils + rbf_compute_weights + rbf_assemble_csr over the
whole node set, inputs resident in HBM.  Default workload: [0,1]^3 minus the
ball B((1/2,1/2,1/2), 0.3), jittered lattice h = 1/106 plus face lattice and
Fibonacci sphere nodes (1,096,553 nodes), n = 35, degree 3 (m = 20), operators
Laplacian, d/dx, d/dy, d/dz.  The reported form is FP32 LU + FP64 refinement;
the plain FP64 form is timed beside it on the same inputs.

    python bench.py [--steps K] [--warmup W] [--form f32_ir|f64] [--no-cpu]

Prints one JSON line.  Only one GPU is supported: --gpus N with N > 1 exits.
"""
from __future__ import annotations

import argparse
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
PEAK_HBM_GBS = 8000.0
OPS = ("lap", "dx", "dy", "dz")


def weights_flops_per_stencil(n: int, m: int, d: int, R: int) -> float:
    """Algorithmic FLOPs of one stencil's weights: LU of the (n+m)^2 system,
    forward/back substitution of R right-hand sides, and the n^2 RBF entries
    (d differences, d squares, d-1 additions, a square root and a product)."""
    M = n + m
    return (2.0 / 3.0) * M ** 3 + 2.0 * R * M * M + (3 * d + 1) * n * n


def knn_bytes_per_stencil(n: int, d: int) -> float:
    """Algorithmic HBM bytes of stencil selection: read the node, write n indices."""
    return 8.0 * d + 4.0 * n


def csr_bytes_per_stencil(n: int, R: int) -> float:
    """Read idx and w, write col and vals, plus the row pointer."""
    return 2.0 * (4.0 * n + 8.0 * R * n) + 8.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", default="f32_ir", choices=["f32_ir", "f64"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-compare", action="store_true", help="time only the reported form")
    ap.add_argument("--cpu-sample", type=int, default=30000)
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed steps, run a plain 1 GiB read + 1 GiB write elementwise kernel "
                         "(torch.neg on float64) three times, the reference for HBM byte counters")
    return ap.parse_args()


# Kernel sources of the weights path; the HBM traffic recorded under profiles/
# belongs to the build whose sources hash to the recorded value.
WEIGHTS_SOURCES = ("include/rbffd.h", "paper_1912_13282_amd/csrc/common.hpp", "paper_1912_13282_amd/csrc/wsolve.hpp",
                   "paper_1912_13282_amd/csrc/weights_kernels.hpp", "paper_1912_13282_amd/csrc/weights.hip",
                   "paper_1912_13282_amd/csrc/wcls_56.hip")
TRAFFIC_FILE = "profiles/traffic_weights_cube_minus_sphere_3d.txt"


def weights_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in WEIGHTS_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(form: str):
    """HBM bytes per launch of the dominant weights kernel from the committed
    FETCH_SIZE / WRITE_SIZE passes, or None if absent or taken on other sources."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != weights_source_hash() or kv.get("form") != form:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    a = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for {max(a.gpus, world)}); "
              "the path shards by node ranges with a halo exchange, which this build does not run.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import nodesets as ns
    import paper_1912_13282_amd as rb

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = ns.workload("cube_sphere3d")
    nd = wl["nodes"][0]
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
    from paper_1912_13282_amd import _binding as B
    ws = torch.empty(B.select_stencils_workspace(N, d, n), dtype=torch.uint8, device=dev)
    w = torch.empty((R, nnz), dtype=torch.float64, device=dev)
    status = torch.empty(N, dtype=torch.int8, device=dev)
    row_ptr = torch.empty(N + 1, dtype=torch.int64, device=dev)
    col = torch.empty(nnz, dtype=torch.int32, device=dev)
    vals = torch.empty((R, nnz), dtype=torch.float64, device=dev)
    ctx = rb.context(dev)
    stream = torch.cuda.current_stream(dev)

    def step(form, evs=None):
        if evs:
            evs[0].record(stream)
        rb.select_stencils(X, offsets, n, idx=idx, workspace=ws, ctx=ctx)
        if evs:
            evs[1].record(stream)
        rb.compute_weights(X, offsets, idx, n, P, ops, precision=form, w=w, status=status, ctx=ctx)
        if evs:
            evs[2].record(stream)
        rb.assemble_csr(offsets, idx, w, n, row_ptr=row_ptr, col=col, vals=vals, ctx=ctx)
        if evs:
            evs[3].record(stream)

    def run_form(form, K, W):
        for _ in range(W):
            step(form)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        wall = time.perf_counter()
        t0.record(stream)
        for k in range(K):
            step(form, evs[k])
        t1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall
        total_ms = t0.elapsed_time(t1)
        ph = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3])] for e in evs])
        st = status.cpu().numpy()
        knn_ms, w_ms, csr_ms = ph.mean(axis=0)
        return dict(form=form, ms_per_step=total_ms / K, wall_ms_per_step=1000.0 * wall / K,
                    phases_ms=dict(select_stencils=knn_ms, compute_weights=w_ms, assemble_csr=csr_ms),
                    stencils_per_s=N / ((total_ms / K) / 1000.0),
                    knn_weights_stencils_per_s=N / ((knn_ms + w_ms) / 1000.0),
                    status_counts={int(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))},
                    fallback_fraction=float(np.mean(st == rb.ST_FALLBACK)))

    results = {}
    forms = [a.form] if a.no_compare else [a.form] + [f for f in ("f64", "f32_ir") if f != a.form]
    weights_snapshot = {}
    for f in forms:
        results[f] = run_form(f, a.steps, a.warmup)
        weights_snapshot[f] = (w.cpu().numpy() if not a.no_cpu else None, idx.cpu().numpy() if f == forms[0] else None)
        print(f"[bench] {f}: {results[f]['ms_per_step']:.3f} ms/step  phases {results[f]['phases_ms']}",
              file=sys.stderr, flush=True)

    main_r = results[a.form]
    flop = weights_flops_per_stencil(n, m, d, R)
    t_w = main_r["phases_ms"]["compute_weights"] / 1000.0
    achieved = flop * N / t_w / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": recorded_traffic(a.form),
                "kernel": "k_weights_ir + k_weights_f64(fallback pass)" if a.form == "f32_ir" else "k_weights_f64",
                "flop_per_stencil": flop, "stencils_per_launch": N}
    phases_roofline = {
        "select_stencils": {"bound": "hbm", "bytes_per_stencil": knn_bytes_per_stencil(n, d),
                            "achieved_GBs": knn_bytes_per_stencil(n, d) * N / (main_r["phases_ms"]["select_stencils"] / 1e3) / 1e9},
        "assemble_csr": {"bound": "hbm", "bytes_per_stencil": csr_bytes_per_stencil(n, R),
                         "achieved_GBs": csr_bytes_per_stencil(n, R) * N / (main_r["phases_ms"]["assemble_csr"] / 1e3) / 1e9},
    }
    for k in phases_roofline:
        phases_roofline[k]["frac"] = phases_roofline[k]["achieved_GBs"] / PEAK_HBM_GBS

    out = {
        "metric": METRIC, "value": main_r["stencils_per_s"], "unit": "stencils/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": main_r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if a.form == "f32_ir" else "f64", "data": "synthetic",
        "config": {"workload": "cube_minus_sphere_3d", "N": N, "nnz": nnz, "n": n, "degree": P, "m": m,
                   "ops": list(ops), "phs_power": 3, "form": a.form,
                   "step": "select_stencils + compute_weights + assemble_csr"},
        "roofline": roofline,
        "phases_roofline": phases_roofline,
        "forms": results,
    }
    if "f64" in results and "f32_ir" in results:
        out["mixed_vs_f64"] = results["f32_ir"]["knn_weights_stencils_per_s"] / results["f64"]["knn_weights_stencils_per_s"]

    if a.calib_copy:
        src = torch.randn(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: 3 x (read {src.numel() * 8} B + write {dst.numel() * 8} B)",
              file=sys.stderr, flush=True)
        del src, dst

    if not a.no_cpu:
        out["cpu_baseline"], out["error"] = cpu_baseline(nd, off, n, P, ops, weights_snapshot, a.cpu_sample)
    print(json.dumps(out), flush=True)


def cpu_baseline(nd, off, n, P, ops, snap, sample_size):
    """The oracle, untuned, on one host core: exact kNN (k-d tree + exact re-rank)
    and weights (one LAPACK gesv per stencil) for a seeded sample of nodes.  The
    same sample also measures the GPU forms' error against the oracle."""
    from threadpoolctl import threadpool_limits

    from oracle import knn as oknn
    from oracle import rbffd as orbf

    rng = np.random.default_rng(12345)
    sample = np.sort(rng.choice(nd.N, size=min(sample_size, nd.N), replace=False))
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        c0 = time.process_time()
        soff, sidx = oknn.knn_exact(nd.X, n, nodes=sample)
        Wo, _ = orbf.weights(nd.X, soff, sidx, P, ops)
        dt = time.perf_counter() - t
        cpu_s = time.process_time() - c0
    st_idx = sidx.reshape(sample.size, n)
    threads = max(1, int(round(cpu_s / dt)))   # threads the oracle kept busy on average
    cpu = {"value": sample.size / dt, "unit": "stencils/s", "cores": threads, "kind": "oracle",
           "sample": f"{sample.size} seeded random nodes of the same workload (kNN against all {nd.N} nodes + weights), "
                     f"{dt:.1f} s wall, {cpu_s:.1f} s CPU, BLAS limited to one thread"}
    # error of each GPU form on the sample (C9-style scaled max-norm)
    err = {}
    h = nd.h[0]
    for f, (wg, ig) in snap.items():
        if wg is None:
            continue
        pos = (off[sample][:, None] + np.arange(n)[None, :]).reshape(-1)
        worst = 0.0
        for c, op in enumerate(ops):
            sc = h ** (2 if op == "lap" else 1)
            den = max(1.0, float(np.max(np.abs(Wo[c]) * sc)))
            worst = max(worst, float(np.max(np.abs(wg[c, pos] - Wo[c]) * sc)) / den)
        err[f] = {"scaled_max_err": worst, "tolerance": 1e-10 if f == "f64" else 1e-9, "sample": int(sample.size)}
    stencils_match = None
    for f, (wg, ig) in snap.items():
        if ig is not None:
            pos = (off[sample][:, None] + np.arange(n)[None, :])
            stencils_match = bool(np.array_equal(ig[pos], st_idx))
    err["stencils_bit_exact_on_sample"] = stencils_match
    return cpu, err


if __name__ == "__main__":
    main()
