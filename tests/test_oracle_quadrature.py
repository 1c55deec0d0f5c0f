"""Pins for the oracle's 1D integrals of eq. Gten_sep: closed forms where the
truncation is negligible or the Gaussian is flat, and mpmath elsewhere."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import psp_oracle as O


def test_gauss_legendre_rule():
    for m in (1, 2, 5, 24, 40):
        x, w = O.gauss_legendre(m)
        xr, wr = np.polynomial.legendre.leggauss(m)
        assert np.allclose(x, xr, atol=1e-15, rtol=0)
        assert np.allclose(w, wr, atol=5e-15, rtol=0)
        # exact for every monomial up to degree 2m-1
        for d in range(2 * m):
            exact = 0.0 if d % 2 else 2.0 / (d + 1)
            assert abs(np.sum(w * x ** d) - exact) < 1e-14


@pytest.mark.parametrize("L", [2.0, 4.0, 8.2])
def test_large_exponent_closed_form(L):
    # alpha (L/2)^2 >= 60: the tail beyond the box is below e^-60 and the
    # integrals equal their full-line values
    n = 24
    a = L / 2
    alphas = np.array([60.0, 300.0, 5e3, 1e6]) / (a * a)
    J0, J2 = O.tables_1d(alphas, n, L)
    k = np.arange(n + 1)
    for s, al in enumerate(alphas):
        xi = 2 * math.pi * k / L
        g = math.sqrt(math.pi / al) * np.exp(-xi * xi / (4 * al))
        j0 = g
        j2 = g * (1.0 / (2 * al)) * (1.0 - xi * xi / (2 * al))
        scale0 = math.sqrt(math.pi / al)
        scale2 = scale0 / (2 * al)
        assert np.max(np.abs(J0[s] - j0)) < 2e-15 * scale0
        assert np.max(np.abs(J2[s] - j2)) < 2e-15 * scale2


@pytest.mark.parametrize("L", [2.0, 4.0])
def test_flat_gaussian_limit(L):
    # alpha -> 0: J0 = L delta_k0, J2(0) = L^3/12, J2(k) = L^3 (-1)^k / (2 pi^2 k^2)
    n = 32
    J0, J2 = O.tables_1d(np.array([1e-30]), n, L)
    k = np.arange(1, n + 1)
    assert abs(J0[0, 0] - L) < 1e-14 * L
    assert np.max(np.abs(J0[0, 1:])) < 1e-14 * L
    assert abs(J2[0, 0] - L ** 3 / 12) < 1e-14 * L ** 3
    want = L ** 3 * (-1.0) ** k / (2 * math.pi ** 2 * k * k)
    assert np.max(np.abs(J2[0, 1:] - want)) < 1e-14 * L ** 3


def test_mpmath_sample():
    mp.mp.dps = 30
    L, n = 4.0, 64
    alphas = np.array([1e-3, 0.07, 0.9, 3.1, 11.0])
    J0, J2 = O.tables_1d(alphas, n, L)
    for s, al in enumerate(alphas):
        for k in (0, 1, 7, 33, 64):
            xi = mp.mpf(2) * mp.pi * k / L
            f0 = lambda y: 2 * mp.exp(-al * y * y) * mp.cos(xi * y)
            f2 = lambda y: 2 * y * y * mp.exp(-al * y * y) * mp.cos(xi * y)
            pts = mp.linspace(0, L / 2, 2 * k + 3)
            v0 = mp.quad(f0, pts)
            v2 = mp.quad(f2, pts)
            scale0 = 2 * mp.quad(lambda y: mp.exp(-al * y * y), [0, L / 2])
            scale2 = 2 * mp.quad(lambda y: y * y * mp.exp(-al * y * y), [0, L / 2])
            # the cosine argument 2 pi k y / L carries a rounding error that
            # grows with k: allow several ulp plus k/2 ulp of the scale
            tol = (8.0 + 0.5 * k) * 1e-16
            assert abs(J0[s, k] - float(v0)) < tol * float(scale0)
            assert abs(J2[s, k] - float(v2)) < tol * float(scale2)


def test_high_wavenumber_value_accuracy():
    # wide Gaussians at high k: the box-truncated integrals are ~k^2 smaller
    # than their integrands; they must still be accurate relative to their
    # own value (the multiplier there is as large as at low k)
    mp.mp.dps = 40
    L, n = 4.8, 48
    alphas = np.array([1e-9, 0.02, 0.4])
    J0, J2 = O.tables_1d(alphas, n, L)
    for s, al in enumerate(alphas):
        for k in (31, 45, 48):
            xi = mp.mpf(2) * mp.pi * k / mp.mpf(L)
            a = mp.mpf(al)
            pts = mp.linspace(0, mp.mpf(L) / 2, 2 * k + 3)
            v0 = mp.quad(lambda y: 2 * mp.exp(-a * y * y) * mp.cos(xi * y), pts)
            v2 = mp.quad(lambda y: 2 * y * y * mp.exp(-a * y * y) * mp.cos(xi * y), pts)
            # value-relative, down to the extended-precision floor of the scale
            assert abs(J0[s, k] - float(v0)) < 5e-14 * abs(float(v0)) + 1e-18 * L, (al, k)
            assert abs(J2[s, k] - float(v2)) < 5e-14 * abs(float(v2)) + 1e-18 * L ** 3, (al, k)


def test_highest_wavenumber_at_full_size():
    # n = 256 (the benchmark size), wide and medium Gaussians at k = n - 1 and
    # n, where the multiplier's sum over Gaussian-sum terms cancels most: the
    # tables must sit far below one ulp of their scale (the exactly reduced
    # cosine phase; phases formed from rounded node positions were ~1e-17 of
    # the scale off at k = n)
    mp.mp.dps = 30
    n = 256
    L = 4.0
    alphas = np.array([4.28e-10, 1.86e-6, 0.536])
    J0, J2 = O.tables_1d(alphas, n, L)
    for s, al in enumerate(alphas):
        a = mp.mpf(al)
        for k in (n - 1, n):
            xi = mp.mpf(2) * mp.pi * k / mp.mpf(L)
            pts = [mp.mpf(0)] + [(j + mp.mpf(0.5)) * mp.mpf(L) / (2 * k) for j in range(k)] + [mp.mpf(L) / 2]
            pts = sorted(p for p in pts if p <= mp.mpf(L) / 2)
            v0 = mp.quad(lambda y: 2 * mp.exp(-a * y * y) * mp.cos(xi * y), pts)
            v2 = mp.quad(lambda y: 2 * y * y * mp.exp(-a * y * y) * mp.cos(xi * y), pts)
            assert abs(J0[s, k] - float(v0)) < 5e-20 * L, (al, k)
            assert abs(J2[s, k] - float(v2)) < 5e-20 * L ** 3 / 12, (al, k)
