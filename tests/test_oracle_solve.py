"""Pins for the oracle's solve (Algorithm 2): the FFT route against the
FFT-free Toeplitz sum, closed forms, the spectral residual and the symmetries
of the discrete operator."""
import math

import numpy as np
import pytest

from oracle import closed_forms as C
from oracle import psp_oracle as O
from paper_2506_04489_amd import densities as D


@pytest.mark.parametrize("n", [4, 8, 12, 16])
def test_fft_route_equals_direct_toeplitz(n):
    # the padded circular convolution never wraps: it IS the Toeplitz sum
    h = 2.0 / n
    rng = np.random.default_rng(n)
    rho = rng.standard_normal((n, n, n))
    su = O.setup(n, h, 40)
    u_fft = O.solve(rho, h, 40, su=su)
    u_dir = O.direct_operator(rho, h, 40, su=su)
    assert np.max(np.abs(u_fft - u_dir)) <= 1e-14 * np.max(np.abs(u_dir))


def test_direct_points_equals_full():
    n, h = 12, 0.17
    rng = np.random.default_rng(3)
    rho = rng.standard_normal((n, n, n))
    su = O.setup(n, h, 40)
    u = O.solve(rho, h, 40, su=su)
    pts = rng.integers(0, n, size=(20, 3))
    got = O.direct_points(rho, pts, h, 40, su=su)
    want = u[pts[:, 0], pts[:, 1], pts[:, 2]]
    assert np.max(np.abs(got - want)) <= 1e-14 * np.max(np.abs(u))


def test_gaussian_closed_form_and_centre_value():
    # rho = exp(-|x|^2/a^2): u = sqrt(pi) a^3 erf(r/a)/(4r), u(0) = a^2/2
    n, a = 64, 0.15
    h = 2.0 / n
    rho = D.gaussian(n, h, -1.0, a)
    xs = -1.0 + h * np.arange(n)
    r = np.sqrt(xs[:, None, None] ** 2 + xs[None, :, None] ** 2 + xs[None, None, :] ** 2)
    u = O.solve(rho, h, 461)
    assert C.relative_max_error(u, C.unnormalised_gaussian_potential(r, a)) < 2e-14
    assert abs(u[n // 2, n // 2, n // 2] - a * a / 2) < 1e-15


def test_spectral_residual_on_crop():
    # -Lap_h u_pad = rho on the original grid (the padding legitimately differs)
    n, a = 64, 0.15
    h = 2.0 / n
    rho = D.gaussian(n, h, -1.0, a)
    up = O.solve_padded(rho, h, 461)
    L = 2 * n * h
    k = np.fft.fftfreq(2 * n, 1.0 / (2 * n))
    K2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    lap = np.fft.ifftn((2 * math.pi / L) ** 2 * K2 * np.fft.fftn(up)).real
    assert np.max(np.abs(lap[:n, :n, :n] - rho)) < 1e-12 * np.max(np.abs(rho))


@pytest.fixture(scope="module")
def small_case():
    n, h = 12, 0.21
    su = O.setup(n, h, 40)
    rng = np.random.default_rng(7)
    return n, h, su, rng


def test_linearity(small_case):
    n, h, su, rng = small_case
    r1, r2 = rng.standard_normal((2, n, n, n))
    a, b = 1.7, -0.3
    lhs = O.solve(a * r1 + b * r2, h, 40, su=su)
    rhs = a * O.solve(r1, h, 40, su=su) + b * O.solve(r2, h, 40, su=su)
    assert np.max(np.abs(lhs - rhs)) <= 1e-14 * np.max(np.abs(lhs))


def test_flips_and_transposes_commute(small_case):
    n, h, su, rng = small_case
    rho = rng.standard_normal((n, n, n))
    u = O.solve(rho, h, 40, su=su)
    scale = np.max(np.abs(u))
    for ax in range(3):
        uf = O.solve(np.flip(rho, ax), h, 40, su=su)
        assert np.max(np.abs(uf - np.flip(u, ax))) <= 1e-14 * scale
    for perm in [(1, 0, 2), (2, 0, 1), (0, 2, 1)]:
        ut = O.solve(np.transpose(rho, perm), h, 40, su=su)
        assert np.max(np.abs(ut - np.transpose(u, perm))) <= 1e-14 * scale


def test_translation_commutes(small_case):
    n, h, su, rng = small_case
    rho = np.zeros((n, n, n))
    rho[2:6, 3:7, 1:5] = rng.standard_normal((4, 4, 4))
    shifted = np.roll(rho, (2, -1, 3), axis=(0, 1, 2))   # support stays inside
    u = O.solve(rho, h, 40, su=su)
    us = O.solve(shifted, h, 40, su=su)
    assert np.max(np.abs(us[2:, :n - 1, 3:] - u[:n - 2, 1:, :n - 3])) <= 1e-14 * np.max(np.abs(u))


def test_positive_density_gives_positive_potential():
    n = 16
    h = 2.0 / n
    rho = D.bump(n, h, -1.0, 0.6)
    u = O.solve(rho, h, 40)
    assert np.all(u > 0)


# ------------------------------------------ continuous references (pins)
def test_oscillatory_matches_heat_semigroup():
    """The oscillatory benchmark density against u = int_0^inf exp(t Lap) rho dt
    (exact up to a 1D trapezoid rule).  With R = 300 the Gaussian sum is
    accurate to about 1e-14 (Section 2, Fig. 1) and the density is resolved
    (a/h = 6.4, w h = 0.63), so the two agree near rounding level; a dropped
    term, sign or factor anywhere in the oracle would show at O(1)."""
    n, R = 64, 300
    h = 2.0 / n
    c = n // 2
    rng = np.random.default_rng(7)
    pts = np.array([(c, c, c), (c + 3, c - 2, c + 1), (c + 5, c, c - 4)]
                   + [tuple(int(v) for v in rng.integers(n // 4, 3 * n // 4, 3)) for _ in range(9)])
    rho = D.oscillatory(n, h, -1.0, a=0.2, omega=20.0)
    got = O.direct_points(rho, pts, h, R)
    ref = C.oscillatory_heat_potential(pts, -1.0, h, 0.2, 20.0)
    e = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    assert e <= 5e-12, e


def test_bump_matches_radial_quadrature_with_spectral_convergence():
    """The C-infinity bump of the headline workload against its radial
    potential (1D quadrature).  The error is the grid's, so it must fall
    faster than any power of h: measured 2.5e-6, 3.6e-7, 3.0e-9 at
    n = 48, 64, 96 (R = 200, below the Gaussian-sum error of 1e-11)."""
    errs = []
    for n in (48, 64, 96):
        h = 2.0 / n
        c = n // 2
        pts = np.array([(c, c, c), (c + 3, c - 2, c + 1), (c + n // 8, c, c - n // 16), (c, c + n // 5, c),
                        (c - n // 4, c - n // 4, c)])
        got = O.direct_points(D.bump(n, h, -1.0, 0.6), pts, h, 200)
        x = -1.0 + h * pts
        ref = C.bump_radial_potential(np.sqrt((x ** 2).sum(axis=1)))
        errs.append(float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
    assert errs[0] <= 1e-5 and errs[1] <= 2e-6 and errs[2] <= 2e-8, errs
    assert errs[1] < errs[0] / 4 and errs[2] < errs[1] / 50, errs
