"""Build libpsp.so (HIP for gfx950 plus host C++) in-tree with hipcc.

Usage: ``python -m paper_2506_04489_amd.build`` or ``build()`` from Python.
Objects go to ``_build/`` at the repository root; the shared library is
written next to this file as ``libpsp.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpsp.so")
BUILD_DIR = os.path.join(ROOT, "_build")
ARCH = "gfx950"

SOURCES = ["passes_f64_lo.hip", "passes_f64_hi.hip", "passes_f32_lo.hip", "passes_f32_hi.hip", "passes_f64_x1.hip",
           "passes_f64_x2.hip", "passes_f32_x1.hip", "passes_f32_x2.hip", "persist_f64.hip",
           "persist_f32.hip", "spectrum.hip", "tables.hip", "peaks.hip", "batched.hip", "noalloc.hip", "setup.cpp", "api.cpp", "serve.cpp", "graph.cpp", "tuning.cpp"]

COMMON = [
    "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]
# every translation unit is compiled as HIP so that host code can use the
# runtime API; device code never uses packed FP32 instructions
HIP_FLAGS = ["-x", "hip", "--offload-arch=" + ARCH,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


# the FFT passes round every instantiation the same way: no automatic
# contraction of a*b+c, the kernels write their fused multiply-adds out
NO_CONTRACT = {"passes_f64_lo.hip", "passes_f64_hi.hip", "passes_f32_lo.hip", "passes_f32_hi.hip",
               "passes_f64_x1.hip", "passes_f64_x2.hip", "passes_f32_x1.hip", "passes_f32_x2.hip",
               "persist_f64.hip", "persist_f32.hip", "tables.hip"}


def _newest_header() -> float:
    heads = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    heads += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    return max(os.path.getmtime(f) for f in heads)


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if t >= os.path.getmtime(os.path.join(CSRC, src)) and t >= _newest_header():
            return obj
    extra = ["-ffp-contract=off"] if src in NO_CONTRACT else []
    cmd = [hipcc()] + HIP_FLAGS + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (with incremental, only those older than their
    object) and link libpsp.so; returns its path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, incremental), srcs))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    sys.exit(0)
