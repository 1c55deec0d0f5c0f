"""S1 on the device (eq. Gten_sep, Algorithm 1 step 1): the 1D tables the
kernel spectrum is built from, against the oracle's independent composite
Gauss-Legendre tables, the full-line closed forms and mpmath at 30 digits,
including the high wavenumbers where the box-truncated integrals are far
below their integrands."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import psp_oracle as O
from paper_2506_04489_amd import psp as B
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


@pytest.mark.parametrize("n,h,R", [(4, 0.5, 40), (32, 2 / 32, 40), (96, 2 / 96, 40), (64, 4 / 63, 120),
                                   (384, 2 / 384, 40), (24, 4 / 23, 461)])
def test_tables_match_oracle(n, h, R):
    p = B.Plan(n, h, R)
    J0, J2 = p.tables()
    _, al = p.gs()
    J0o, J2o = O.tables_1d(al, n, 2 * n * h)
    # both sides carry ~1e-19 of the scale before the final rounding (the
    # oracle's extended-precision phases ~1e-18 at k ~ 384): every entry
    # agrees to 1e-15 of itself plus 4e-18 of its row's scale
    worst = 0.0
    for s in range(R):
        for J, Jo in ((J0, J0o), (J2, J2o)):
            sc = max(np.max(np.abs(Jo[s])), 1e-300)
            excess = np.abs(J[s] - Jo[s]) - 1e-15 * np.abs(Jo[s])
            worst = max(worst, float(np.max(excess)) / sc)
    print("n=%d R=%d max (|J - J_oracle| - 1e-15 |J_oracle|) / scale %.2e" % (n, R, worst))
    assert worst <= 4e-18


def test_closed_form_rows():
    # the narrow Gaussians take the full-line closed forms; against the same
    # forms in 30-digit arithmetic (J2 changes sign where xi^2 = 2a)
    n, h, R = 128, 2 / 128, 40
    L = 2 * n * h
    p = B.Plan(n, h, R)
    J0, J2 = p.tables()
    _, al = p.gs()
    rows = [s for s in range(R) if al[s] * (L / 2) ** 2 >= 50]
    assert rows
    mp.mp.dps = 30
    for s in rows:
        a = mp.mpf(al[s])
        ref0, ref2 = [], []
        for k in range(n + 1):
            xi = 2 * mp.pi * k / L
            e = mp.sqrt(mp.pi / a) * mp.exp(-xi * xi / (4 * a))
            ref0.append(float(e))
            ref2.append(float(e * (2 * a - xi * xi) / (4 * a * a)))
        ref0, ref2 = np.array(ref0), np.array(ref2)
        assert np.all(np.abs(J0[s] - ref0) <= 1e-15 * np.abs(ref0)), s
        assert np.all(np.abs(J2[s] - ref2) <= 1e-15 * np.abs(ref2) + 1e-18 * np.max(np.abs(ref2))), s


def _mp_table(a, L, k, p):
    mp.mp.dps = 30
    a, L = mp.mpf(a), mp.mpf(L)
    xi = 2 * mp.pi * k / L
    f = lambda y: y ** p * mp.exp(-a * y * y) * mp.cos(xi * y)
    b = L / 2
    pts = [b * i / (2 * k + 8) for i in range(2 * k + 9)]
    return 2 * mp.quad(f, pts)


def test_high_wavenumbers_against_mpmath():
    # the widest Gaussians, whose box-truncated integrals at k ~ n are ~n^2
    # below their integrands: every sample to 1e-14 relative, or, where the
    # value is itself tiny, to 1e-18 of the row's scale
    n, h, R = 256, 2 / 256, 40
    L = 2 * n * h
    p = B.Plan(n, h, R)
    J0, J2 = p.tables()
    _, al = p.gs()
    for s in (0, 3, 12, 20):
        assert al[s] * (L / 2) ** 2 < 50            # quadrature rows
        for k in (0, 1, 37, n // 2, n - 1, n):
            for pw, J in ((0, J0), (2, J2)):
                ref = float(_mp_table(al[s], L, k, pw))
                scale = float(np.max(np.abs(J[s])))
                err = abs(J[s][k] - ref)
                assert err <= 1e-18 * scale or err <= 1e-14 * abs(ref), (s, k, pw, J[s][k], ref)


def test_tables_deterministic_and_precompute_consistent():
    n, h, R = 64, 2 / 64, 40
    p = B.Plan(n, h, R)
    a0, a2 = p.tables()
    b0, b2 = p.tables()
    assert np.array_equal(a0, b0) and np.array_equal(a2, b2)
    p.precompute()
    c0, c2 = p.tables()
    assert np.array_equal(a0, c0) and np.array_equal(a2, c2)


def test_device_peaks_are_plausible():
    pk = B.device_peaks(1 << 28)
    print("measured peaks", pk)
    assert 500 < pk["copy_GBps"] < 8000          # below the 8 TB/s HBM3E spec
    assert 5 < pk["fp64_mfma_TFLOPs"] < 78.6     # below the FP64 MFMA spec
