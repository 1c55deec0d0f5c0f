"""Loader of the oracle's C naive FFT (``oracle/naive_fft.c``).

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only the tests, the smoke
check and the CPU-baseline leg of the benchmark reach this module (through
``psp_oracle``).  The library is built with gcc next to its source the first
time it is needed (or by ``build()``), without fast-math and without
floating-point contraction, with OpenMP over the independent lines.
"""
from __future__ import annotations

import ctypes
import os
import shutil
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "naive_fft.c")
LIB = os.path.join(HERE, "libnaive_fft.so")
FLAGS = ["-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11"]

_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile naive_fft.c into libnaive_fft.so (when missing, older than the
    source, or with force); returns the library path."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        raise RuntimeError("no C compiler found for the oracle's FFT")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [cc] + FLAGS + ["-o", tmp, SRC, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("oracle FFT build failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            path = build()
            L = ctypes.CDLL(path)
            L.oracle_fft_axis.restype = ctypes.c_int
            L.oracle_fft_axis.argtypes = [ctypes.c_void_p, ctypes.c_long, ctypes.c_long, ctypes.c_long,
                                          ctypes.c_int, ctypes.c_int]
            L.oracle_set_threads.restype = ctypes.c_int
            L.oracle_set_threads.argtypes = [ctypes.c_int]
            _lib = L
    return _lib


def set_threads(t: int) -> int:
    """Threads of the C FFT's later calls (t <= 0: the OpenMP default);
    returns the count in force."""
    return int(lib().oracle_set_threads(int(t)))


def fft_axis_inplace(a: np.ndarray, axis: int, sign: int) -> None:
    """Unnormalised DFT along ``axis`` of a C-contiguous complex128 3D array,
    in place (sign -1 forward, +1 inverse)."""
    if a.dtype != np.complex128 or a.ndim != 3 or not a.flags.c_contiguous:
        raise ValueError("need a C-contiguous complex128 3D array")
    rc = lib().oracle_fft_axis(a.ctypes.data, a.shape[0], a.shape[1], a.shape[2], int(axis), int(sign))
    if rc == -1:
        raise ValueError("length %d is not a product of 2s and 3s" % a.shape[axis])
    if rc != 0:
        raise MemoryError("oracle FFT ran out of memory")
