"""Build the HIP library librbffd.so for gfx950 in-tree (hipcc, no JIT cache).

    python -m paper_1912_13282_amd.build [--jobs N] [--verbose]

Every .hip file under csrc/ is compiled to an object in _build/ and linked into
paper_1912_13282_amd/librbffd.so.  Always recompiles (the build check must see
every source).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "librbffd.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    # packed FP32 VALU forms are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the 128-step eliminations must unroll completely (register arrays are
    # indexed by the step), which is above LLVM's default size limit
    "-mllvm", "-pragma-unroll-threshold=1000000",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def compile_one(src: str, verbose: bool, extra: list[str]) -> tuple[str, float, str]:
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    # -save-temps routes the device code through the assembler, which rejects any
    # instruction the target cannot encode instead of letting it be emitted silently
    cmd = [HIPCC, *FLAGS, "-save-temps=obj", *extra, "-c", src, "-o", obj]
    t = time.time()
    p = subprocess.run(cmd, capture_output=True, text=True)
    out = (p.stdout + p.stderr)
    # the host pass does not know the packed-fp32 feature; that note is harmless
    out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")
    return obj, time.time() - t, out if verbose else ""


def _stale(src: str) -> bool:
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    if not os.path.exists(obj):
        return True
    deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    deps.append(os.path.join(ROOT, "include", "rbffd.h"))
    return max(os.path.getmtime(f) for f in deps) > os.path.getmtime(obj)


def build(jobs: int | None = None, verbose: bool = False, extra: list[str] | None = None,
          incremental: bool = False) -> str:
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(BUILD, exist_ok=True)
    extra = list(extra or [])
    srcs = sources()
    todo = [s for s in srcs if _stale(s)] if incremental else srcs
    jobs = jobs or max(1, min(8, os.cpu_count() or 4, len(todo)))
    objs = [os.path.join(BUILD, os.path.basename(s)[:-4] + ".o") for s in srcs]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for obj, dt, out in ex.map(lambda s: compile_one(s, verbose, extra), todo):
            if verbose:
                print(f"  {os.path.basename(obj)}: {dt:.1f}s")
                if out:
                    print(out)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout + p.stderr)
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--incremental", action="store_true", help="recompile only sources newer than their objects")
    ap.add_argument("--resource-usage", action="store_true",
                    help="print per-kernel VGPR/SGPR/LDS/spill usage")
    a = ap.parse_args(argv)
    extra = ["-Rpass-analysis=kernel-resource-usage"] if a.resource_usage else []
    t = time.time()
    lib = build(a.jobs, a.verbose or a.resource_usage, extra, incremental=a.incremental)
    print(f"built {lib} in {time.time() - t:.1f}s")


if __name__ == "__main__":
    sys.exit(main())
