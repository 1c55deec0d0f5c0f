"""Exact potentials for the paper's benchmark densities (test infrastructure).

TEST INFRASTRUCTURE: imported only by the tests, the smoke check and the
benchmark's CPU leg.  Each pair (rho, u*) satisfies ``-Lap u* = rho`` with
``u* -> 0``; where the paper prints rho, the formula here is ``-Lap u*``
derived from the printed u* (and checked symbolically in the tests).

  * normalised Gaussian and its erf potential (Section 3.2, eq. gaussian);
  * two superposed Gaussians (eq. gaussians);
  * anisotropic Gaussian u* (eq. anis);
  * oscillating u* = exp(-r^2/s^2) cos(w r^2) (eq. osci).  The printed rho
    carries ``-4 w^2 r^2 cos(w r^2)``; ``-Lap u*`` has ``+4 w^2 r^2 cos``;
  * bump u* = exp(-d/(1 - r^2/R^2)) (eq. bump).  The printed rho's exponent and
    its ``-d R^2 r^2`` term do not match u*; ``-Lap u*`` is
    ``2 d R^2 (3R^4 - 2R^2 r^2 - r^4 - 2 d R^2 r^2)/(R^2 - r^2)^4
    exp(-d R^2/(R^2 - r^2))``;
  * the benchmark's oscillatory density through the heat semigroup, and its
    C-infinity bump through the radial potential integral (1D quadratures).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def paper_grid(N: int, lo: float = -2.0, hi: float = 2.0):
    """The paper's node grid: N points per axis including both box ends,
    spacing ``(hi - lo)/(N - 1)``.  Returns (h, X, Y, Z) broadcastable."""
    h = (hi - lo) / (N - 1)
    xs = lo + h * np.arange(N)
    return h, xs[:, None, None], xs[None, :, None], xs[None, None, :]


def erf_potential(r, sigma):
    """Potential of the unit-mass Gaussian of standard deviation sigma:
    ``erf(r/(sqrt(2) sigma)) / (4 pi r)``, with its limit at r = 0."""
    r = np.asarray(r, dtype=np.float64)
    safe = np.where(r > 0, r, 1.0)
    val = erf(safe / (math.sqrt(2.0) * sigma)) / (4.0 * math.pi * safe)
    return np.where(r > 0, val, math.sqrt(2.0 / math.pi) / (4.0 * math.pi * sigma))


def gaussian_pair(X, Y, Z, sigma, centre=(0.0, 0.0, 0.0)):
    r = np.sqrt((X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2)
    rho = np.exp(-r * r / (2.0 * sigma * sigma)) / ((2.0 * math.pi) ** 1.5 * sigma ** 3)
    return rho, erf_potential(r, sigma)


def unnormalised_gaussian_potential(r, a):
    """Potential of ``exp(-|x|^2/a^2)``: ``sqrt(pi) a^3 erf(r/a) / (4 r)``,
    equal to ``a^2/2`` at r = 0."""
    r = np.asarray(r, dtype=np.float64)
    safe = np.where(r > 0, r, 1.0)
    val = math.sqrt(math.pi) * a ** 3 * erf(safe / a) / (4.0 * safe)
    return np.where(r > 0, val, 0.5 * a * a)


def two_gaussians_pair(X, Y, Z, d=(0.1, -0.05, 0.05), s1=0.2, s2=0.1):
    r1, u1 = gaussian_pair(X, Y, Z, s1, d)
    r2, u2 = gaussian_pair(X, Y, Z, s2, tuple(-v for v in d))
    return 0.5 * (r1 + r2), 0.5 * (u1 + u2)


def anisotropic_pair(X, Y, Z, sig=(0.30, 0.20, 0.28), c=(0.0, 0.0, 0.0)):
    sx, sy, sz = sig
    dx, dy, dz = X - c[0], Y - c[1], Z - c[2]
    u = np.exp(-dx ** 2 / sx ** 2 - dy ** 2 / sy ** 2 - dz ** 2 / sz ** 2)
    rho = -(4 * dx ** 2 / sx ** 4 + 4 * dy ** 2 / sy ** 4 + 4 * dz ** 2 / sz ** 4
            - 2 / sx ** 2 - 2 / sy ** 2 - 2 / sz ** 2) * u
    return rho, u


def oscillating_pair(X, Y, Z, sigma=0.3, omega=20.0, c=(0.0, 0.0, 0.0)):
    g = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2
    e = np.exp(-g / sigma ** 2)
    u = e * np.cos(omega * g)
    rho = (e * (6 * omega * np.sin(omega * g) + 4 * omega ** 2 * g * np.cos(omega * g))
           - (4 * g / sigma ** 4 - 6 / sigma ** 2) * e * np.cos(omega * g)
           - 8 * omega * g / sigma ** 2 * e * np.sin(omega * g))
    return rho, u


def oscillating_rho_as_printed(X, Y, Z, sigma=0.3, omega=20.0):
    """eq. osci exactly as printed (with ``-4 w^2 r^2 cos``), for the test that
    shows it does not reproduce the paper's own error table."""
    g = X ** 2 + Y ** 2 + Z ** 2
    e = np.exp(-g / sigma ** 2)
    return (e * (6 * omega * np.sin(omega * g) - 4 * omega ** 2 * g * np.cos(omega * g))
            - (4 * g / sigma ** 4 - 6 / sigma ** 2) * e * np.cos(omega * g)
            - 8 * omega * g / sigma ** 2 * e * np.sin(omega * g))


def bump_pair(X, Y, Z, d=10.0, R=2.0, c=(0.0, 0.0, 0.0)):
    r2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2
    inside = r2 < R * R
    den = np.where(inside, R * R - r2, 1.0)
    e = np.where(inside, np.exp(-d * R * R / den), 0.0)
    u = e
    rho = np.where(inside, 2 * d * R ** 2 * (3 * R ** 4 - 2 * R ** 2 * r2 - r2 ** 2
                                            - 2 * d * R ** 2 * r2) / den ** 4 * e, 0.0)
    return rho, u


def relative_max_error(u, u_ref):
    """The paper's E: max |u - u_h| / max |u| over the grid (eq. error_infty)."""
    return float(np.max(np.abs(u - u_ref)) / np.max(np.abs(u_ref)))


def cube_abs_integral(a: float) -> float:
    """``int_{[-a,a]^3} |y| dy``: by symmetry 8 octants, each 3 times the
    region where y1 is the largest coordinate; with ``y2 = y1 s, y3 = y1 t``
    that region gives ``int_0^a y1^3 dy1 * I = a^4 I / 4``, so the total is
    ``6 a^4 I`` with the smooth ``I = int_0^1 int_0^1 sqrt(1 + s^2 + t^2) ds dt``
    (mpmath, 30 digits)."""
    import mpmath as mp
    mp.mp.dps = 30
    I = mp.quad(lambda s, t: mp.sqrt(1 + s * s + t * t), [0, 1], [0, 1])
    return float(6 * mp.mpf(a) ** 4 * I)


def oscillatory_heat_potential(points, x0, h, a=0.2, omega=20.0, s_lo=-40.0, s_hi=12.0, m=6001):
    """u at grid indices ``points`` (P, 3) for the density
    ``exp(-|x|^2/a^2) sin(w x1) cos(w x2) sin(w x3)`` on the grid
    ``x = x0 + j h``, from the heat semigroup: with -Lap u = rho and u -> 0,
    ``u = int_0^inf (exp(t Lap) rho) dt``.  rho is a product of 1D factors
    ``exp(-x^2/a^2) exp(i w x)`` (imaginary part for sin, real part for
    cos), and the 1D heat flow maps that factor to
    ``sqrt(a^2/(a^2+4t)) exp(-(x - i w a^2/2)^2/(a^2+4t) - w^2 a^2/4)``.
    The t integral is a trapezoid rule in s = ln t on [s_lo, s_hi], where the
    integrand is negligible at both ends."""
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    x = x0 + h * pts
    s = np.linspace(s_lo, s_hi, m)
    t = np.exp(s)[None, :]
    d = a * a + 4.0 * t

    def flow(xp):
        z = xp[:, None] - 0.5j * omega * a * a
        return np.sqrt(a * a / d) * np.exp(-z * z / d - omega * omega * a * a / 4.0)

    g = flow(x[:, 0]).imag * flow(x[:, 1]).real * flow(x[:, 2]).imag * t
    ds = (s_hi - s_lo) / (m - 1)
    return ds * (g.sum(axis=1) - 0.5 * (g[:, 0] + g[:, -1]))


def bump_radial_potential(r, radius=0.6):
    """The potential of the radial bump ``exp(-1/(1 - s^2/R^2))`` (s < R):
    ``u(r) = (1/r) int_0^r s^2 rho(s) ds + int_r^R s rho(s) ds``, the
    exterior-shell and interior-ball contributions of 1/(4 pi |x - y|), by
    adaptive quadrature (relative tolerance 1e-13)."""
    from scipy.integrate import quad

    def rho(s):
        q = 1.0 - (s / radius) ** 2
        return math.exp(-1.0 / q) if q > 0 else 0.0

    out = []
    for rv in np.atleast_1d(np.asarray(r, dtype=np.float64)):
        rc = min(rv, radius)
        inner = quad(lambda s: s * s * rho(s), 0.0, rc, epsabs=0.0, epsrel=1e-13, limit=400)[0] if rc > 0 else 0.0
        outer = quad(lambda s: s * rho(s), rc, radius, epsabs=0.0, epsrel=1e-13, limit=400)[0] if rc < radius else 0.0
        out.append(inner / rv + outer if rv > 0 else outer)
    return np.array(out)


def gaussian_laplacian(X, Y, Z, sigma, centre=(0.0, 0.0, 0.0)):
    """Laplacian of the normalised Gaussian of ``gaussian_pair``:
    ``rho (r^2/sigma^4 - 3/sigma^2)``."""
    r2 = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2
    rho = np.exp(-r2 / (2.0 * sigma * sigma)) / ((2.0 * math.pi) ** 1.5 * sigma ** 3)
    return rho * (r2 / sigma ** 4 - 3.0 / sigma ** 2)


def gs_cutoff_moment(omega, alpha, r_cut):
    """Mass of the super-potential kernel's cutoff defect (Lemma 1 and its
    proof, Section 2): ``M0 = int_{|y| < r_cut} (|y|/(8 pi) - V_GS(y)) dy``
    with ``V_GS(r) = r^2 sum_s w_s exp(-a_s r^2)`` (eq. gs_x).

    The defect lives in the ball of radius ~eps where the Gaussian sum stops
    following 1/r; beyond it the two kernels agree to the fit error, so any
    r_cut of a few eps gives the same M0.  For a smooth density the
    super-potential v = V * rho is then off by ``M0 rho(x) + O(eps^6)``, and
    since U = Lap V the potential u = Lap v is off by
    ``u_h - u = -M0 Lap rho(x) + O(eps^6)``: the O(eps^4) law of the
    error bound (Theorem 1).  Composite 24-point Gauss-Legendre on panels
    split at the Gaussian widths 1/sqrt(a_s)."""
    w = np.asarray(omega, dtype=np.float64)
    a = np.asarray(alpha, dtype=np.float64)
    x, wt = np.polynomial.legendre.leggauss(24)
    widths = sorted(float(1.0 / math.sqrt(v)) for v in a if 1.0 / math.sqrt(v) < r_cut)
    edges = [0.0] + widths + [r_cut]
    total = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        for k in range(4):
            l = lo + (hi - lo) * k / 4.0
            r = lo + (hi - lo) * (k + 1) / 4.0
            y = 0.5 * (l + r) + 0.5 * (r - l) * x
            vgs = y * y * (np.exp(-np.outer(y * y, a)) @ w)
            total += 0.5 * (r - l) * float(np.sum(wt * 4.0 * math.pi * y * y * (y / (8.0 * math.pi) - vgs)))
    return total


def box_grid(N: int, box):
    """The paper's node grid on a rectangular box ((lo, hi) per axis): N
    points per axis including both ends.  Returns (h, X, Y, Z) with h the
    three spacings ``(hi - lo)/(N - 1)`` and X, Y, Z broadcastable."""
    hs = tuple((hi - lo) / (N - 1) for lo, hi in box)
    xs = [lo + h * np.arange(N) for (lo, _), h in zip(box, hs)]
    return hs, xs[0][:, None, None], xs[1][None, :, None], xs[2][None, None, :]


def box_pair(family: str, params: str, box, X, Y, Z):
    """(rho, u*) of the paper's rectangular-box benchmarks at the box centre:
    'gauss' (sigma), 'bump' ("R/d"), 'anis' (L: sigma = (0.2, 0.2 L, 0.2 L))."""
    c = tuple(0.5 * (lo + hi) for lo, hi in box)
    if family == "gauss":
        return gaussian_pair(X, Y, Z, float(params), c)
    if family == "bump":
        R, d = (float(v) for v in params.split("/"))
        return bump_pair(X, Y, Z, d, R, c)
    if family == "anis":
        L = float(params)
        return anisotropic_pair(X, Y, Z, (0.2, 0.2 * L, 0.2 * L), c)
    raise KeyError(family)
