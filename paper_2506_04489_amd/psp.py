"""Thin ctypes binding of libpsp (the C ABI in include/psp.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  PyTorch provides device memory and streams.  If libpsp.so has not
been built, importing works but the first call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsp.so")

PSP_F64, PSP_F32 = 0, 1
STATUS = {0: "PSP_OK", -1: "PSP_EINVAL", -2: "PSP_ENOMEM", -3: "PSP_EUNSUPPORTED",
          -4: "PSP_ESTATE", -5: "PSP_EHIP", -6: "PSP_EBUSY",
          -7: "PSP_ECANCELED"}

# every entry point the header declares, with (restype, argtypes)
_vp, _i, _d, _sz, _u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_uint64
_P = ctypes.POINTER
SIGNATURES = {
    "psp_plan_create": (_i, [_i, _d, _i, _i, _P(_vp)]),
    "psp_plan_create_ex": (_i, [_i, _d, _i, _i, _d, _d, _P(_vp)]),
    "psp_plan_create_box": (_i, [_i, _P(_d), _i, _i, _d, _d, _P(_vp)]),
    "psp_plan_create_grid": (_i, [_P(_i), _P(_d), _i, _i, _d, _d, _P(_vp)]),
    "psp_device_peaks": (_i, [_vp, _vp, _sz, _vp, _P(_d), _P(_d)]),
    "psp_kernel_precompute": (_i, [_vp, _vp]),
    "psp_solve": (_i, [_vp, _vp, _vp, _vp]),
    "psp_solve_noalloc": (_i, [_vp, _vp, _vp, _vp]),
    "psp_solve_batched": (_i, [_i, _P(_vp), _P(_vp), _P(_vp), _vp]),
    "psp_set_batch_mode": (_i, [_i]),
    "psp_solve_padded_debug": (_i, [_vp, _vp, _vp, _vp]),
    "psp_plan_get_gs": (_i, [_vp, _P(_d), _P(_d)]),
    "psp_debug_guards": (_i, [_i]),
    "psp_plan_check_guards": (_i, [_vp, _P(_i)]),
    "psp_plan_get_tables": (_i, [_vp, _P(_d), _P(_d)]),
    "psp_plan_get_multiplier": (_i, [_vp, _P(_d)]),
    "psp_plan_workspace_bytes": (_i, [_vp, _P(_sz)]),
    "psp_plan_spectrum_bytes": (_i, [_vp, _P(_sz)]),
    "psp_plan_destroy": (None, [_vp]),
    "psp_profile_enable": (_i, [_vp, _i]),
    "psp_plan_set_tuning": (_i, [_vp, _i, _i]),
    "psp_plan_set_shape": (_i, [_vp, _P(_i), _P(_i)]),
    "psp_plan_get_shape": (_i, [_vp, _P(_i), _P(_i)]),
    "psp_tuning_set": (_i, [_i, _i, _P(_i), _P(_i)]),
    "psp_tuning_get": (_i, [_i, _i, _P(_i), _P(_i)]),
    "psp_autotune": (_i, [_vp, _i, _vp, _P(_i), _P(_i), _P(ctypes.c_float), _P(ctypes.c_float)]),
    "psp_profile_read": (_i, [_vp, _P(_i), _P(_d)]),
    "psp_graph_capture": (_i, [_vp, _vp, _vp, _vp, _P(_vp)]),
    "psp_graph_capture_batched": (_i, [_i, _P(_vp), _P(_vp), _P(_vp), _vp, _P(_vp)]),
    "psp_graph_launch": (_i, [_vp, _vp]),
    "psp_graph_destroy": (None, [_vp]),
    "psp_serve_create": (_i, [_sz, _i, _P(_vp)]),
    "psp_serve_submit": (_i, [_vp, _i, _d, _i, _i, _vp, _vp, _P(_u64)]),
    "psp_serve_poll": (_i, [_vp, _u64, _P(_i), _P(_i), _P(_d)]),
    "psp_serve_cancel": (_i, [_vp, _u64]),
    "psp_serve_drain": (_i, [_vp]),
    "psp_serve_stats": (_i, [_vp, _P(_sz), _P(_sz), _P(_u64), _P(_u64), _P(_u64)]),
    "psp_serve_destroy": (None, [_vp]),
    "psp_strerror": (ctypes.c_char_p, [_i]),
    "psp_last_error": (ctypes.c_char_p, []),
}

_lib = None


class PspError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__("%s: %s" % (STATUS.get(status, status), detail))


def lib() -> ctypes.CDLL:
    """Load libpsp.so once; raise if it is missing (no CPU fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpsp.so is not built (run paper_2506_04489_amd.build.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        _load_shipped_tuning()
    return _lib


def _check(status: int):
    if status != 0:
        raise PspError(status, lib().psp_last_error().decode())


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dtype_code(dtype) -> int:
    if dtype in ("f64", "float64", PSP_F64):
        return PSP_F64
    if dtype in ("f32", "float32", PSP_F32):
        return PSP_F32
    import torch
    if dtype is torch.float64:
        return PSP_F64
    if dtype is torch.float32:
        return PSP_F32
    raise ValueError("dtype must be f64 or f32")


def _torch_dtype(code: int):
    import torch
    return torch.float64 if code == PSP_F64 else torch.float32


def _ints5(v):
    v = [int(x) for x in v]
    if len(v) != 5:
        raise ValueError("a shape has 5 entries (passes H1..H5)")
    return (ctypes.c_int * 5)(*v)


def device_peaks(nbytes: int = 1 << 30, stream=None):
    """psp_device_peaks on two scratch tensors of nbytes each: the measured
    streaming-copy rate (GB/s, read plus write) and FP64 MFMA rate
    (TFLOP/s) of the current device."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    gbps, tflops = ctypes.c_double(), ctypes.c_double()
    torch.cuda.synchronize()
    _check(lib().psp_device_peaks(a.data_ptr(), b.data_ptr(), nbytes, _stream_ptr(stream), ctypes.byref(gbps),
                                  ctypes.byref(tflops)))
    return {"copy_GBps": gbps.value, "fp64_mfma_TFLOPs": tflops.value}


def debug_guards(enable: bool):
    """Workspaces allocated from now on sit between pattern-filled guard bands."""
    _check(lib().psp_debug_guards(1 if enable else 0))


def set_batch_mode(mode: str):
    """'grouped' (default): one launch per pass per (n, shape); 'persistent':
    persistent kernels over every solve with 2n <= 256; 'flat': the same
    kernels with one workgroup per work item."""
    codes = {"grouped": 0, "persistent": 1, "flat": 2}
    if mode not in codes:
        raise ValueError("mode must be 'grouped', 'persistent' or 'flat'")
    _check(lib().psp_set_batch_mode(codes[mode]))


def tuning_set(n: int, dtype, plan, tile):
    """Enter a launch shape for (n, dtype) in the process-wide tuning table."""
    _check(lib().psp_tuning_set(int(n), _dtype_code(dtype), _ints5(plan), _ints5(tile)))


def tuning_get(n: int, dtype):
    pa, ta = (ctypes.c_int * 5)(), (ctypes.c_int * 5)()
    _check(lib().psp_tuning_get(int(n), _dtype_code(dtype), pa, ta))
    return list(pa), list(ta)


TUNING_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")


def load_tuning(path: str) -> int:
    """Load a tuning table written by ``paper_2506_04489_amd.autotune``;
    returns the number of entries entered."""
    import json
    with open(path) as f:
        doc = json.load(f)
    count = 0
    for e in doc.get("entries", []):
        tuning_set(e["n"], e["dtype"], e["plan"], e["tile"])
        count += 1
    return count


def _load_shipped_tuning():
    # PSP_TUNING_FILE names another table; "none" keeps the default shapes
    path = os.environ.get("PSP_TUNING_FILE", TUNING_FILE)
    if path and path != "none" and os.path.exists(path):
        load_tuning(path)


class Plan:
    """One (n, h, R, dtype) configuration: psp_plan_create[_ex] + helpers.
    h is one spacing, or three (one per axis: a rectangular box,
    psp_plan_create_box); n is one point count, or three (one per axis,
    psp_plan_create_grid; rho is then n[0] x n[1] x n[2] and ``n`` holds
    n[0])."""

    def __init__(self, n, h, R: int, dtype="f64", eps: float = None, delta: float = None):
        self.R = int(R)
        self.code = _dtype_code(dtype)
        handle = ctypes.c_void_p()
        if np.ndim(n) > 0:
            if len(list(n)) != 3:
                raise ValueError("n must be one point count or three")
            self.shape3 = tuple(int(v) for v in n)
            self.n = self.shape3[0]
            hl = [float(v) for v in (h if np.ndim(h) > 0 else (h, h, h))]
            if len(hl) != 3:
                raise ValueError("h must be one spacing or three")
            self.h = tuple(hl)
            ns = (ctypes.c_int * 3)(*self.shape3)
            hs = (ctypes.c_double * 3)(*self.h)
            _check(lib().psp_plan_create_grid(ns, hs, self.R, self.code, -1.0 if eps is None else float(eps),
                                              -1.0 if delta is None else float(delta), ctypes.byref(handle)))
            self._h = handle
            return
        self.n = int(n)
        self.shape3 = (self.n,) * 3
        if np.ndim(h) > 0:
            if len(list(h)) != 3:
                raise ValueError("h must be one spacing or three")
            self.h = tuple(float(v) for v in h)
            hs = (ctypes.c_double * 3)(*self.h)
            _check(lib().psp_plan_create_box(self.n, hs, self.R, self.code, -1.0 if eps is None else float(eps),
                                             -1.0 if delta is None else float(delta), ctypes.byref(handle)))
        elif eps is None and delta is None:
            self.h = float(h)
            _check(lib().psp_plan_create(self.n, self.h, self.R, self.code, ctypes.byref(handle)))
        else:
            self.h = float(h)
            _check(lib().psp_plan_create_ex(self.n, self.h, self.R, self.code, float(eps), float(delta),
                                            ctypes.byref(handle)))
        self._h = handle

    @property
    def handle(self):
        return self._h

    @property
    def torch_dtype(self):
        return _torch_dtype(self.code)

    def close(self):
        if self._h:
            lib().psp_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def precompute(self, stream=None):
        _check(lib().psp_kernel_precompute(self._h, _stream_ptr(stream)))
        return self

    def _check_tensor(self, t, shape):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise ValueError("expected a CUDA (HIP) tensor")
        if t.dtype != self.torch_dtype:
            raise ValueError("tensor dtype %s does not match the plan's %s" % (t.dtype, self.torch_dtype))
        if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError("expected a contiguous tensor of shape %s" % (shape,))

    def solve(self, rho, u=None, stream=None):
        import torch
        self._check_tensor(rho, self.shape3)
        if u is None:
            u = torch.empty_like(rho)
        self._check_tensor(u, self.shape3)
        _check(lib().psp_solve(self._h, rho.data_ptr(), u.data_ptr(), _stream_ptr(stream)))
        return u

    def solve_noalloc(self, rho, u, stream=None):
        """psp_solve_noalloc: the solve with its intermediates in the
        library's fixed device array; u must be given (nothing is allocated)."""
        self._check_tensor(rho, self.shape3)
        self._check_tensor(u, self.shape3)
        _check(lib().psp_solve_noalloc(self._h, rho.data_ptr(), u.data_ptr(), _stream_ptr(stream)))
        return u

    def solve_padded_debug(self, rho, stream=None):
        import torch
        self._check_tensor(rho, self.shape3)
        up = torch.empty(tuple(2 * v for v in self.shape3), dtype=rho.dtype, device=rho.device)
        _check(lib().psp_solve_padded_debug(self._h, rho.data_ptr(), up.data_ptr(), _stream_ptr(stream)))
        return up

    def gs(self):
        om = np.empty(self.R)
        al = np.empty(self.R)
        _check(lib().psp_plan_get_gs(self._h, om.ctypes.data_as(_P(_d)), al.ctypes.data_as(_P(_d))))
        return om, al

    def tables(self):
        J0 = np.empty((self.R, self.n + 1))
        J2 = np.empty((self.R, self.n + 1))
        _check(lib().psp_plan_get_tables(self._h, J0.ctypes.data_as(_P(_d)), J2.ctypes.data_as(_P(_d))))
        return J0, J2

    def multiplier(self):
        m = np.empty(tuple(v + 1 for v in self.shape3))
        _check(lib().psp_plan_get_multiplier(self._h, m.ctypes.data_as(_P(_d))))
        return m

    def set_tuning(self, k3_tiles: int = 0, i1_group: int = 0):
        _check(lib().psp_plan_set_tuning(self._h, int(k3_tiles), int(i1_group)))
        return self

    def set_shape(self, plan, tile):
        """Launch shape of passes H1..H5: radix plan and tile choice per pass."""
        pa, ta = _ints5(plan), _ints5(tile)
        _check(lib().psp_plan_set_shape(self._h, pa, ta))
        return self

    def guards_intact(self) -> bool:
        """psp_plan_check_guards: the guard bands of this plan's workspaces
        (allocated while psp_debug_guards was on) are untouched."""
        ok = ctypes.c_int()
        _check(lib().psp_plan_check_guards(self._h, ctypes.byref(ok)))
        return bool(ok.value)

    def shape(self):
        """(plan[5], tile[5]) of this plan."""
        pa, ta = (ctypes.c_int * 5)(), (ctypes.c_int * 5)()
        _check(lib().psp_plan_get_shape(self._h, pa, ta))
        return list(pa), list(ta)

    def autotune(self, reps: int = 5, stream=None):
        """Time every candidate shape of every pass (psp_autotune); the plan
        and the process-wide tuning table take the fastest.  Returns
        {"plan": [...], "tile": [...], "pass_ms": [...], "candidates_ms": [[...] x 5]}
        where candidates_ms[i][plan * 21 + tile] is each candidate's
        time (-1: no such candidate)."""
        pa, ta = (ctypes.c_int * 5)(), (ctypes.c_int * 5)()
        ms = (ctypes.c_float * 5)()
        cm = (ctypes.c_float * 315)()
        _check(lib().psp_autotune(self._h, int(reps), _stream_ptr(stream), pa, ta, ms, cm))
        cand = [[round(float(cm[i * 63 + c]), 5) for c in range(63)] for i in range(5)]
        return {"plan": list(pa), "tile": list(ta), "pass_ms": [float(x) for x in ms], "candidates_ms": cand}

    def profile_enable(self, max_solves: int):
        _check(lib().psp_profile_enable(self._h, int(max_solves)))

    def profile_read(self):
        """(count, [ms of passes H1..H5], ms of the whole solve)."""
        cnt = ctypes.c_int()
        ms = np.zeros(6)
        _check(lib().psp_profile_read(self._h, ctypes.byref(cnt), ms.ctypes.data_as(_P(_d))))
        return cnt.value, ms[:5].tolist(), float(ms[5])

    def workspace_bytes(self) -> int:
        v = ctypes.c_size_t()
        _check(lib().psp_plan_workspace_bytes(self._h, ctypes.byref(v)))
        return v.value

    def spectrum_bytes(self) -> int:
        v = ctypes.c_size_t()
        _check(lib().psp_plan_spectrum_bytes(self._h, ctypes.byref(v)))
        return v.value


def solve_batched(plans: Sequence[Plan], rhos, us, stream=None):
    """psp_solve_batched over matching lists of plans, inputs and outputs."""
    k = len(plans)
    if not (len(rhos) == k and len(us) == k):
        raise ValueError("plans, rhos and us must have the same length")
    for p, r, u in zip(plans, rhos, us):
        p._check_tensor(r, p.shape3)
        p._check_tensor(u, p.shape3)
    ph = (ctypes.c_void_p * k)(*[p.handle.value for p in plans])
    rp = (ctypes.c_void_p * k)(*[r.data_ptr() for r in rhos])
    up = (ctypes.c_void_p * k)(*[u.data_ptr() for u in us])
    _check(lib().psp_solve_batched(k, ph, rp, up, _stream_ptr(stream)))
    return us


class Graph:
    """A solve (or batch) captured as a HIP graph: psp_graph_*."""

    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep            # tensors and plans the graph points into

    @classmethod
    def capture(cls, plan: "Plan", rho, u, stream=None):
        plan._check_tensor(rho, plan.shape3)
        plan._check_tensor(u, plan.shape3)
        h = ctypes.c_void_p()
        _check(lib().psp_graph_capture(plan.handle, rho.data_ptr(), u.data_ptr(), _stream_ptr(stream),
                                       ctypes.byref(h)))
        return cls(h, (plan, rho, u))

    @classmethod
    def capture_batched(cls, plans, rhos, us, stream=None):
        k = len(plans)
        for p, r, u in zip(plans, rhos, us):
            p._check_tensor(r, p.shape3)
            p._check_tensor(u, p.shape3)
        ph = (ctypes.c_void_p * k)(*[p.handle.value for p in plans])
        rp = (ctypes.c_void_p * k)(*[r.data_ptr() for r in rhos])
        up = (ctypes.c_void_p * k)(*[u.data_ptr() for u in us])
        h = ctypes.c_void_p()
        _check(lib().psp_graph_capture_batched(k, ph, rp, up, _stream_ptr(stream), ctypes.byref(h)))
        return cls(h, (list(plans), list(rhos), list(us)))

    def launch(self, stream=None):
        _check(lib().psp_graph_launch(self._h, _stream_ptr(stream)))

    def close(self):
        if self._h:
            lib().psp_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """psp_serve_*: the continuous-batching request loop."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 64):
        h = ctypes.c_void_p()
        _check(lib().psp_serve_create(int(hbm_budget_bytes), int(max_slots), ctypes.byref(h)))
        self._h = h

    def submit(self, n, h, R, tier, rho, u) -> int:
        t = ctypes.c_uint64()
        _check(lib().psp_serve_submit(self._h, int(n), float(h), int(R), _dtype_code(tier),
                                      rho.data_ptr(), u.data_ptr(), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        done = ctypes.c_int()
        res = ctypes.c_int()
        lat = ctypes.c_double()
        _check(lib().psp_serve_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(done), ctypes.byref(res),
                                    ctypes.byref(lat)))
        return bool(done.value), res.value, lat.value

    def cancel(self, ticket: int) -> bool:
        """Withdraw a queued request (True); False if it is already on the
        device and will complete normally."""
        st = lib().psp_serve_cancel(self._h, ctypes.c_uint64(ticket))
        if st == -6:
            return False
        _check(st)
        return True

    def drain(self):
        _check(lib().psp_serve_drain(self._h))

    def stats(self):
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        c, d, e = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().psp_serve_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d),
                                     ctypes.byref(e)))
        return {"bytes_in_use": a.value, "bytes_peak": b.value, "completed": c.value, "cache_hits": d.value,
                "cache_misses": e.value}

    def close(self):
        if self._h:
            lib().psp_serve_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
