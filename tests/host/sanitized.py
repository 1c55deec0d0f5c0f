"""Host build of libpsp with AddressSanitizer and UndefinedBehaviorSanitizer
(test infrastructure).

The library's host sources are compiled with ``-Xarch_host -fsanitize=...``
(device code, where present, is compiled as usual and is not instrumented);
the FFT pass instantiations and persistent batch kernels are replaced by
``pass_stubs.hip``.  ``abi_driver.c`` (instrumented too) then drives the C
ABI's host logic, and ``oracle_fft_driver.c`` the oracle's C FFT built with
gcc's sanitizers.  Objects go to ``_build/sanitized``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2506_04489_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "sanitized")
LIB_SOURCES = ["spectrum.hip", "tables.hip", "peaks.hip", "batched.hip", "noalloc.hip", "setup.cpp", "api.cpp",
               "serve.cpp", "graph.cpp", "tuning.cpp"]
HIP_SAN = ["-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-fno-omit-frame-pointer", "-fPIC", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include")]
ROCM = "/opt/rocm"


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("%s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))


def hipcc():
    return os.environ.get("HIPCC") or shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")


def build_library() -> str:
    os.makedirs(OUT, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in LIB_SOURCES] + [os.path.join(HERE, "pass_stubs.hip")]

    def one(src):
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        _run([hipcc()] + HIP_SAN + ["-c", src, "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(one, srcs))
    lib = os.path.join(OUT, "libpsp_san.so")
    _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
          "-Xarch_host", "-fsanitize=undefined", "-o", lib] + objs + ["-lpthread"])
    return lib


def build_abi_driver() -> str:
    lib = build_library()
    exe = os.path.join(OUT, "abi_driver")
    clang = os.path.join(ROCM, "llvm", "bin", "clang")
    _run([clang, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "abi_driver.c"), "-o", exe,
          "-L", OUT, "-lpsp_san", "-Wl,-rpath," + os.path.dirname(lib),
          "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    return exe


def build_oracle_driver() -> str:
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_fft_driver")
    _run(["gcc", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-ffp-contract=off", os.path.join(ROOT, "oracle", "naive_fft.c"), os.path.join(HERE, "oracle_fft_driver.c"),
          "-o", exe, "-lm"])
    return exe
