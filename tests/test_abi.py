"""The C ABI without a GPU: exported symbols, argument validation, and the
host-side precompute (Gaussian-sum fit and 1D integrals) against the oracle's
independent implementations."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import psp_oracle as O
from paper_2506_04489_amd import psp as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "psp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(psp_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(B.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(B.SIGNATURES)


@pytest.mark.parametrize("n,h,R,code", [
    (31, 0.1, 40, "PSP_EUNSUPPORTED"),    # odd n
    (10, 0.1, 40, "PSP_EUNSUPPORTED"),    # 2n = 20 has a factor 5
    (2, 0.1, 40, "PSP_EUNSUPPORTED"),     # too small
    (512, 0.1, 40, "PSP_EUNSUPPORTED"),   # above the supported maximum
    (30, 0.1, 40, "PSP_EUNSUPPORTED"),    # 2n = 60 has a factor 5
    (486, 0.1, 40, "PSP_EUNSUPPORTED"),   # 2n = 972 = 4 * 3^5, above 384
    (32, 0.0, 40, "PSP_EINVAL"),
    (32, -1.0, 40, "PSP_EINVAL"),
    (32, float("inf"), 40, "PSP_EINVAL"),
    (32, float("nan"), 40, "PSP_EINVAL"),
    (32, 0.1, 0, "PSP_EINVAL"),
    (32, 0.1, 5000, "PSP_EINVAL"),
])
def test_plan_create_rejects(n, h, R, code):
    with pytest.raises(B.PspError) as ei:
        B.Plan(n, h, R)
    assert B.STATUS[ei.value.status] == code


def test_every_2a3b_size_is_accepted():
    # Algorithm 1 takes any grid size: every even n in [4, 384] with
    # 2n = 2^a 3^b gets a plan, every other n in that range is refused
    def smooth(m):
        while m % 2 == 0:
            m //= 2
        while m % 3 == 0:
            m //= 3
        return m == 1
    for n in range(4, 385, 2):
        if smooth(2 * n):
            p = B.Plan(n, 2.0 / n, 8)
            assert p.workspace_bytes() > 0
            p.close()
        else:
            with pytest.raises(B.PspError) as ei:
                B.Plan(n, 2.0 / n, 8)
            assert B.STATUS[ei.value.status] == "PSP_EUNSUPPORTED"


def test_plan_create_ex_rejects_bad_cutoff():
    with pytest.raises(B.PspError) as ei:
        B.Plan(32, 0.1, 40, eps=2.0, delta=1.0)
    assert B.STATUS[ei.value.status] == "PSP_EINVAL"


@pytest.mark.parametrize("h,eps,delta,code", [
    ((0.1, 0.0, 0.1), None, None, "PSP_EINVAL"),             # a zero spacing
    ((0.1, -0.2, 0.1), None, None, "PSP_EINVAL"),
    ((0.1, float("nan"), 0.1), None, None, "PSP_EINVAL"),
    ((0.1, 0.2, 0.3), 2.0, 1.0, "PSP_EINVAL"),                # eps > delta
    ((0.1, 0.2, 0.3), 1e-4, float("inf"), "PSP_EINVAL"),
])
def test_box_plan_rejects(h, eps, delta, code):
    with pytest.raises(B.PspError) as ei:
        B.Plan(32, h, 40, eps=eps, delta=delta)
    assert B.STATUS[ei.value.status] == code


def test_box_plan_create_null_and_defaults():
    lib = B.lib()
    out = ctypes.c_void_p()
    assert B.STATUS[lib.psp_plan_create_box(32, None, 40, 0, -1.0, -1.0, ctypes.byref(out))] == "PSP_EINVAL"
    assert not out.value
    with pytest.raises(ValueError):
        B.Plan(32, (0.1, 0.2), 40)
    # default cutoff: 1e-4 of the longest half side, delta the half diagonal,
    # i.e. the oracle's; equal spacings give the cubic plan's Gaussian sum
    hs = (0.05, 0.08, 0.11)
    p = B.Plan(32, hs, 40)
    eps, delta = O.default_eps_delta(32, hs)
    wo, ao = O.gs_weights(40, eps, delta)
    w, a = p.gs()
    assert np.allclose(w, wo, rtol=1e-14, atol=0) and np.allclose(a, ao, rtol=1e-14, atol=0)
    q, c = B.Plan(32, (0.1, 0.1, 0.1), 40), B.Plan(32, 0.1, 40)
    assert all(np.array_equal(x, y) for x, y in zip(q.gs(), c.gs()))


def test_grid_plan_create_validation_and_layout():
    lib = B.lib()
    out = ctypes.c_void_p()
    h3 = (ctypes.c_double * 3)(0.1, 0.1, 0.1)
    assert B.STATUS[lib.psp_plan_create_grid(None, h3, 40, 0, -1.0, -1.0, ctypes.byref(out))] == "PSP_EINVAL"
    for bad in [(32, 31, 32), (32, 10, 32), (32, 32, 512), (2, 32, 32)]:
        with pytest.raises(B.PspError) as ei:
            B.Plan(bad, 0.1, 40)
        assert B.STATUS[ei.value.status] == "PSP_EUNSUPPORTED", bad
    ns, hs = (16, 24, 32), (0.1, 0.2, 0.3)
    p = B.Plan(ns, hs, 40)
    assert p.shape3 == ns and p.n == 16
    eps, delta = O.default_eps_delta(ns, hs)
    wo, ao = O.gs_weights(40, eps, delta)
    w, a = p.gs()
    assert np.allclose(w, wo, rtol=1e-14, atol=0) and np.allclose(a, ao, rtol=1e-14, atol=0)
    # every pass takes the tuned shape of a cube of its own axis's size
    plan, tile = p.shape()
    for q, m in enumerate((32, 24, 16, 24, 32)):
        tp, tt = B.tuning_get(m, "f64")
        assert (plan[q], tile[q]) == (tp[q], tt[q]), q
    pitch = lambda m: ((m + 1 + 15) // 16) * 16
    cols = lambda m: ((m + 1 + 7) // 8) * 8
    assert p.workspace_bytes() == 16 * (pitch(32) * 16 * 24 + 16 * a_plane(16, 24, cols(32), 16))
    assert p.spectrum_bytes() == 8 * 17 * 25 * pitch(32)
    # equal counts: the box plan
    q, c = B.Plan((16, 16, 16), hs, 40), B.Plan(16, hs, 40)
    assert all(np.array_equal(x, y) for x, y in zip(q.gs(), c.gs()))
    assert q.shape() == c.shape()
    for call in (lambda: p.set_shape([0] * 5, [0] * 5), lambda: p.set_tuning(2, 0), lambda: p.profile_enable(1)):
        with pytest.raises(B.PspError) as ei:
            call()
        assert B.STATUS[ei.value.status] == "PSP_EUNSUPPORTED"


def test_error_strings():
    lib = B.lib()
    for code in B.STATUS:
        assert lib.psp_strerror(code)
    with pytest.raises(B.PspError):
        B.Plan(31, 0.1, 40)
    assert b"even" in lib.psp_last_error()


def test_solve_before_precompute_is_state_error():
    p = B.Plan(16, 0.125, 40)
    st = B.lib().psp_solve(p.handle, ctypes.c_void_p(16), ctypes.c_void_p(32), None)
    assert B.STATUS[st] == "PSP_ESTATE"
    st = B.lib().psp_solve(p.handle, None, ctypes.c_void_p(32), None)
    assert B.STATUS[st] == "PSP_EINVAL"


@pytest.mark.parametrize("n,h,R", [(32, 2 / 32, 40), (128, 2 / 128, 40), (64, 4 / 63, 461), (24, 0.3, 7)])
def test_gs_weights_match_oracle(n, h, R):
    p = B.Plan(n, h, R)
    om, al = p.gs()
    eps, delta = O.default_eps_delta(n, h)
    om_o, al_o = O.gs_weights(R, eps, delta)
    # same published formula, two implementations: agreement to a few ulp
    assert np.max(np.abs(om / om_o - 1)) < 1e-15 * max(1, R / 40)
    assert np.max(np.abs(al / al_o - 1)) < 1e-14 * max(1, R / 40)


def a_plane(n1, n2, pa, elem):
    """i1 pitch (elements) of a chunk buffer of n1 planes of 2 n2 rows of pa
    columns: above 128 MiB the smallest whole number of 128-byte lines that
    holds a plane and is 15 mod 32 lines (so that the fused i1 pass's column
    reads spread over the HBM channels), else the plane itself."""
    need = 2 * n2 * pa * elem
    assert need % 128 == 0
    lines = need // 128
    if need * n1 > 128 << 20:
        while lines % 32 != 15:
            lines += 1
    return lines * 128 // elem


def test_chunk_plane_pitch():
    assert a_plane(256, 256, 264, 16) == 256 * 2 * 264 + 15 * 8   # n = 256 FP64: 15 lines of pad
    assert a_plane(128, 128, 136, 16) == 256 * 136                # 71 MB: no pad
    for n in (2, 3, 12, 24, 96, 128, 192, 256, 384):
        for pa, elem in ((8, 16), (16, 8), (264, 16), (272, 8), (392, 16)):
            pl = a_plane(n, n, pa, elem)
            assert 2 * n * pa <= pl < 2 * n * pa + 32 * 128 // elem


def test_workspace_and_spectrum_sizes():
    # X: n*n*P complex; chunk buffer: n planes of 2n rows of tiles*W complex
    # (W = 8 FP64 or 16 FP32 k3 bins per tile; by default one chunk of all
    # tiles), the plane pitch padded as a_plane says
    p = B.Plan(256, 2 / 256, 40)
    P = 272
    assert p.workspace_bytes() == 16 * (P * 256 * 256 + 256 * a_plane(256, 256, 264, 16))
    assert p.spectrum_bytes() == 8 * 257 * 257 * P
    q = B.Plan(256, 2 / 256, 40, dtype="f32")
    assert q.workspace_bytes() == 8 * (P * 256 * 256 + 256 * a_plane(256, 256, 272, 8))
    p.set_tuning(4, 0)
    assert p.workspace_bytes() == 16 * (P * 256 * 256 + 256 * a_plane(256, 256, 32, 16))


# ---------------------------------------------------------------- shapes
def test_shape_validation_and_roundtrip():
    p = B.Plan(32, 2 / 32, 40)                       # 2n = 64: no alternative radix plans
    assert p.shape() == B.tuning_get(32, "f64")      # new plans start from the table
    p.set_shape([0] * 5, [2, 1, 2, 1, 1])
    assert p.shape() == ([0] * 5, [2, 1, 2, 1, 1])
    p.set_shape([0] * 5, [0, 0, 20, 0, 0])           # H3: tile 6 with nontemporal loads and stores
    assert p.shape() == ([0] * 5, [0, 0, 20, 0, 0])
    p.set_shape([0] * 5, [0, 13, 0, 9, 0])           # H2, H4: tiles 6 and 2 with nontemporal A accesses
    assert p.shape() == ([0] * 5, [0, 13, 0, 9, 0])
    p.set_shape([0] * 5, [7, 0, 0, 0, 4])            # H1, H5: nontemporal stores
    assert p.shape() == ([0] * 5, [7, 0, 0, 0, 4])
    for plan, tile in [([1, 0, 0, 0, 0], [0] * 5),   # no alternative plan for 2n = 64
                       ([0] * 5, [8, 0, 0, 0, 0]),   # four workgroup sizes for H1, two cache policies
                       ([0] * 5, [0, 0, 0, 0, 8]),   # and for H5
                       ([0] * 5, [0, 14, 0, 0, 0]),  # fourteen for H2 (two cache policies)
                       ([0] * 5, [0, 0, 0, 14, 0]),  # and for H4
                       ([0] * 5, [0, 0, 21, 0, 0]),  # twenty-one for H3 (three cache policies)
                       ([0] * 5, [0, 0, 0, 0, -1])]:
        with pytest.raises(B.PspError) as ei:
            p.set_shape(plan, tile)
        assert B.STATUS[ei.value.status] == "PSP_EINVAL"
    q = B.Plan(64, 2 / 64, 40)                       # 2n = 128 has both alternatives
    q.set_shape([1, 1, 1, 1, 1], [0] * 5)
    assert q.shape()[0] == [1] * 5
    q.set_shape([2, 2, 2, 2, 2], [0] * 5)
    r = B.Plan(96, 2 / 96, 40)                       # 2n = 192: radix 16 but no plan 1
    r.set_shape([2] * 5, [0] * 5)
    with pytest.raises(B.PspError):
        r.set_shape([1] * 5, [0] * 5)
    with pytest.raises(B.PspError):
        q.set_shape([3] * 5, [0] * 5)
    with pytest.raises(ValueError):
        q.set_shape([0] * 4, [0] * 5)


def test_tuning_table_seeds_new_plans(tmp_path):
    import json
    old = B.tuning_get(96, "f32")
    try:
        B.tuning_set(96, "f32", [0] * 5, [1, 0, 1, 0, 2])
        assert B.tuning_get(96, "f32") == ([0] * 5, [1, 0, 1, 0, 2])
        assert B.Plan(96, 2 / 96, 40, dtype="f32").shape() == ([0] * 5, [1, 0, 1, 0, 2])
        assert B.Plan(96, 2 / 96, 40, dtype="f64").shape() == B.tuning_get(96, "f64")
        with pytest.raises(B.PspError):
            B.tuning_set(10, "f64", [0] * 5, [0] * 5)
        path = tmp_path / "t.json"
        path.write_text(json.dumps({"entries": [{"n": 96, "dtype": "f32", "plan": [0] * 5,
                                                 "tile": [2, 1, 0, 1, 0], "pass_ms": [0] * 5}]}))
        assert B.load_tuning(str(path)) == 1
        assert B.tuning_get(96, "f32") == ([0] * 5, [2, 1, 0, 1, 0])
    finally:
        B.tuning_set(96, "f32", *old)


def test_shipped_tuning_table_is_valid():
    import json
    if not os.path.exists(B.TUNING_FILE):
        pytest.skip("no tuning table shipped")
    doc = json.load(open(B.TUNING_FILE))
    seen = set()
    for e in doc["entries"]:
        key = (e["n"], e["dtype"])
        assert key not in seen
        seen.add(key)
        assert B.tuning_get(e["n"], e["dtype"]) == (e["plan"], e["tile"])


def test_batch_mode_validation():
    lib = B.lib()
    assert lib.psp_set_batch_mode(3) == -1         # PSP_EINVAL
    assert lib.psp_set_batch_mode(-1) == -1
    with pytest.raises(ValueError):
        B.set_batch_mode("fast")
    B.set_batch_mode("persistent")
    B.set_batch_mode("flat")
    B.set_batch_mode("grouped")


def test_empty_batch_is_a_no_op():
    assert B.lib().psp_solve_batched(0, None, None, None, None) == 0


# ------------------------------------------------- 1D-table quadrature rule
def test_gauss_kronrod_constants_are_exact():
    """The 15-point Gauss-Kronrod rule the device tables use (the nodes and
    weights written out in tables.hip): exact for polynomials up to degree
    22 to ~1e-30, and of no higher degree; its odd-position nodes are the
    7-point Gauss nodes, the roots of P_7."""
    import re
    import mpmath as mp
    src = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "paper_2506_04489_amd", "csrc", "tables.hip")).read()

    def arr(name):
        body = re.search(r"%s\[8\] = \{(.*?)\};" % name, src, re.S).group(1)
        return [mp.mpf(v) for v in re.findall(r"([0-9.]+)L", body)]

    mp.mp.dps = 40
    x, w = arr("kXgk"), arr("kWgk")
    assert len(x) == 8 and len(w) == 8 and x[7] == 0
    nodes = [-v for v in x[:7]] + [mp.mpf(0)] + list(reversed(x[:7]))
    wts = w[:7] + [w[7]] + list(reversed(w[:7]))
    for d in range(0, 23):
        got = mp.fsum(wi * xi ** d for wi, xi in zip(wts, nodes))
        want = mp.mpf(2) / (d + 1) if d % 2 == 0 else mp.mpf(0)
        assert abs(got - want) < mp.mpf("1e-30"), d
    for v in (x[1], x[3], x[5], x[7]):
        assert abs(mp.legendre(7, v)) < mp.mpf("1e-30")
    # degree 24 is not integrated exactly (the rule is not of higher degree)
    got = mp.fsum(wi * xi ** 24 for wi, xi in zip(wts, nodes))
    assert abs(got - mp.mpf(2) / 25) > mp.mpf("1e-12")


def test_device_peaks_rejects_bad_arguments():
    lib = B.lib()
    g, t = ctypes.c_double(), ctypes.c_double()
    assert B.STATUS[lib.psp_device_peaks(None, None, 1 << 20, None, ctypes.byref(g), ctypes.byref(t))] == "PSP_EINVAL"
    buf = ctypes.c_void_p(4096)          # never dereferenced: the size check comes first
    assert B.STATUS[lib.psp_device_peaks(buf, buf, 1000, None, ctypes.byref(g), ctypes.byref(t))] == "PSP_EINVAL"
