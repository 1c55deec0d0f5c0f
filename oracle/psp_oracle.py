"""CPU FP64 oracle for the super-potential Gaussian-sum FFT Poisson solve.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this module.  It shares no code with the GPU
library: its own Gaussian-sum construction, its own Gauss-Legendre 1D
quadrature, a plain triple loop for the kernel spectrum, its own naive
recursive mixed-radix (2 and 3) FFT (in numpy, fft_naive, and the same
recursion in plain C, naive_fft.c, which the solve uses by default so that
whole grids up to n = 384 finish in seconds), and a direct (FFT-free)
evaluation of the discrete convolution operator.  Everything is float64,
except the 1D integral sums, which run in extended precision (see
tables_1d).

The method (Exl & Schaffer, "Near-field-free super-potential FFT method for
the three-dimensional free-space Poisson equation"):

  * the free-space problem ``-Lap u = rho`` on R^3 with ``u -> 0`` (Section 1,
    eq. problem1) has ``u = U * rho`` with ``U = 1/(4 pi |x|)`` (eq. conv);
  * ``u = Lap v`` with ``v = V * rho`` and the biharmonic kernel
    ``V(y) = |y|/(8 pi)`` (eq. superpot, superpot1);
  * rho is zero-padded by a factor 2 per axis, so the periodic box has side
    ``L = 2 n h`` and the kernel is truncated to ``[-L/2, L/2]^3``
    (Section 2, eq. conv2 and the Fourier series that follows it);
  * ``u = -(2 pi/L)^2 sum_k |k|^2 Vhat_k rhohat_k e^{2 pi i k.x/L}``
    (eq. convtheorem, written for a general period L instead of L = 2);
  * ``Vhat_k`` is the Fourier integral of V over the truncation box
    (eq. Gten0), replaced by that of the Gaussian-sum approximation
    ``V_GS(y) = |y|^2 sum_s w_s exp(-a_s |y|^2)`` (eq. sin_1_x, gs_x), which
    separates into products of 1D integrals (eq. Gten_sep);
  * the solve is Algorithm 2: FFT of the padded rho, multiply, inverse FFT,
    crop; the precompute is Algorithm 1.

Readings of points the paper leaves open (each also listed in the design
notes of the repository):

  * Sinc quadrature (Section 2 after the Gamma-integral identity): the
    substitution ``t = e^u`` in ``1/r = (2/sqrt(pi)) int_0^inf e^{-r^2 t^2} dt``
    and the trapezoid rule in u with R nodes ``u_s = u0 + s*tau``.  The step
    tau and offset u0 are fixed, not fitted, by balancing three error
    estimates at a common level ``eta = e^{-x}``: discretisation
    ``exp(-pi^2/(2 tau))``, left truncation at ``r = delta`` and right
    truncation at ``r = eps``; x solves ``(R-1) tau = u_max - u0`` by a fixed
    100-step bisection on [1, 80].
  * ``eps = 1e-4 * L/2`` (the paper's default cutoff in units where L = 2) and
    ``delta = sqrt(3) * L/2`` (the corner of the truncation box).
  * Rectangular domains (Section 3, Tables 4, 6, 8; Algorithm 1 takes a
    point count and a spacing per axis): n_p points and spacing h_p on axis
    p, so the padded box has sides ``L_p = 2 n_p h_p``;
    the kernel is truncated to that box, the 1D integrals of axis p run over
    ``[-L_p/2, L_p/2]``, the spectral Laplacian is
    ``-(2 pi)^2 sum_p k_p^2 / L_p^2``, ``eps = 1e-4 max_p(L_p/2)`` and
    ``delta = |(L_1, L_2, L_3)|/2``.
  * The 1D integrals run over the full truncation interval ``[-L/2, L/2]``.
  * The DFT normalisation ``1/(2n)^3`` and the factor ``-(2 pi/L)^2`` are
    folded into one real multiplier per wavenumber.
"""
from __future__ import annotations

import concurrent.futures as _futures
import math
import os

import numpy as np

__all__ = [
    "spacings", "counts", "default_eps_delta", "gs_parameters", "gs_weights", "gs_biharmonic",
    "gauss_legendre", "tables_1d", "spectrum_octant", "multiplier_octant",
    "fft_naive", "fftn_naive", "fftn_c", "solve", "solve_padded", "direct_operator",
    "direct_points", "Setup", "setup",
]

# --------------------------------------------------------------------------
# Algorithm 1, step 1: Gaussian-sum weights and exponents (Section 2,
# eq. sin_1_x and gs_x).
# --------------------------------------------------------------------------


def spacings(h):
    """(h_1, h_2, h_3) from one spacing (cubic cells) or three."""
    hs = tuple(float(v) for v in np.atleast_1d(h))
    if len(hs) == 1:
        return hs * 3
    if len(hs) != 3:
        raise ValueError("h must be one spacing or three")
    return hs


def counts(n):
    """(n_1, n_2, n_3) from one point count per axis (a cube) or three."""
    ns = tuple(int(v) for v in np.atleast_1d(n))
    if len(ns) == 1:
        return ns * 3
    if len(ns) != 3:
        raise ValueError("n must be one point count or three")
    return ns


def default_eps_delta(n, h):
    """Cutoff eps and outer radius delta for n points per axis (one count,
    or one per axis) of spacing h (one value, or one per axis)."""
    halves = [m * v for m, v in zip(counts(n), spacings(h))]   # L_p/2 with L_p = 2 n_p h_p
    return 1e-4 * max(halves), math.sqrt(sum(v * v for v in halves))


def _count_fn(x: float, eps: float, delta: float) -> float:
    # number of trapezoid steps needed to span [u0, u_max] at error level e^-x
    tau = math.pi ** 2 / (2.0 * x)
    u0 = -x - math.log(2.0 * delta / math.sqrt(math.pi))
    umax = math.log(math.sqrt(x) / eps)
    return (umax - u0) / tau


def gs_parameters(R: int, eps: float, delta: float):
    """Trapezoid step tau and first node u0 for an R-term sinc quadrature of
    1/r on (eps, delta] (sinc quadrature, Section 2)."""
    if R < 1:
        raise ValueError("R must be >= 1")
    target = float(R - 1)
    lo, hi = 1.0, 80.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if _count_fn(mid, eps, delta) > target:
            hi = mid
        else:
            lo = mid
    x = lo
    tau = math.pi ** 2 / (2.0 * x)
    u0 = -x - math.log(2.0 * delta / math.sqrt(math.pi))
    return tau, u0


def gs_weights(R: int, eps: float, delta: float):
    """Weights w_s and exponents a_s, s = 0..R-1, with
    ``1/(8 pi r) ~= sum_s w_s exp(-a_s r^2)`` on (eps, delta] (eq. sin_1_x).

    From ``1/r = (2/sqrt(pi)) int exp(-r^2 e^{2u} + u) du`` the trapezoid
    rule gives ``a_s = e^{2 u_s}`` and ``w_s = tau e^{u_s} / (4 pi^{3/2})``.
    """
    tau, u0 = gs_parameters(R, eps, delta)
    omega = np.empty(R)
    alpha = np.empty(R)
    c = tau / (4.0 * math.pi ** 1.5)
    for s in range(R):
        u = u0 + s * tau
        alpha[s] = math.exp(2.0 * u)
        omega[s] = c * math.exp(u)
    return omega, alpha


def gs_biharmonic(r, omega, alpha):
    """``V_GS(r) = r^2 sum_s w_s exp(-a_s r^2)`` (eq. gs_x), elementwise in r."""
    r = np.asarray(r, dtype=np.float64)
    r2 = r * r
    acc = np.zeros_like(r2)
    for w, a in zip(omega, alpha):
        acc += w * np.exp(-a * r2)
    return r2 * acc


# --------------------------------------------------------------------------
# Algorithm 1, step 2: 1D integrals of eq. Gten_sep by composite
# Gauss-Legendre quadrature, then the tensor assembly by a plain loop.
# --------------------------------------------------------------------------


def gauss_legendre(m: int, dtype=np.float64):
    """Nodes and weights of the m-point Gauss-Legendre rule on [-1, 1],
    by Newton iteration on the three-term Legendre recurrence, in ``dtype``."""
    one = dtype(1)
    x = np.cos(math.pi * (np.arange(1, m + 1) - 0.25) / (m + 0.5)).astype(dtype)
    tol = 4 * np.finfo(dtype).eps

    def legendre(x):
        p0 = np.ones_like(x)
        p1 = x.copy()
        for k in range(2, m + 1):
            p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
        dp = m * (x * p1 - p0) / (x * x - one)
        return p1, dp

    for _ in range(100):
        p1, dp = legendre(x)
        dx = p1 / dp
        x = x - dx
        if np.max(np.abs(dx)) < tol:
            break
    p1, dp = legendre(x)
    w = 2 * one / ((one - x * x) * dp * dp)
    order = np.argsort(x)
    return x[order], w[order]


_GL_POINTS = 24
_LD = np.longdouble


def tables_1d(alpha, n: int, L: float):
    """``J0[s,k] = int_{-L/2}^{L/2} exp(-a_s y^2) cos(2 pi k y / L) dy`` and
    ``J2[s,k] = int_{-L/2}^{L/2} y^2 exp(-a_s y^2) cos(2 pi k y / L) dy`` for
    k = 0..n (eq. Gten_sep with the period L in place of 2).

    Both integrands are even in y, so the integral is twice the one over
    [0, b] with ``b = min(L/2, 9/sqrt(a_s))`` (beyond 9/sqrt(a) the Gaussian
    is below e^-81).  The interval is split into equal panels no wider than
    ``min(L/(2n+2), 1/sqrt(a_s))`` (a fraction of the shortest cosine period
    and of the Gaussian width) with a 24-point Gauss-Legendre rule on each.

    The sums run in x87 extended precision (numpy longdouble) and are rounded
    to float64 at the end: for wide Gaussians the box-truncated integrals at
    high k are ~k^2 smaller than the integrand, so float64 node positions and
    cosine arguments alone would leave ~1e-12 relative errors there.  Where
    the interval is the whole half box (b = L/2) the cosine's phase is
    reduced exactly by its integer part (see the code).
    """
    alpha = np.asarray(alpha, dtype=np.float64)
    xg, wg = gauss_legendre(_GL_POINTS, _LD)
    Ll = _LD(L)
    two_pi = 2 * np.arccos(_LD(-1))
    k = np.arange(n + 1).astype(_LD)
    J0 = np.empty((alpha.size, n + 1))
    J2 = np.empty((alpha.size, n + 1))

    t = (1 + xg) / 2                      # node offsets within a panel, in panel widths
    kint = np.arange(n + 1, dtype=np.int64)

    def row(s):
        a = _LD(alpha[s])
        b = min(Ll / 2, _LD(9) / np.sqrt(a))
        width = min(Ll / (2 * n + 2), 1 / np.sqrt(a), b)
        panels = int(math.ceil(float(b / width) - 1e-12))
        j = np.arange(panels)
        y = (b * (j[:, None] + t[None, :]) / panels).ravel()     # node j + t of panel j
        wy = np.tile(wg, panels) * (b / (2 * panels))
        g = np.exp(-a * y * y) * wy
        if b == Ll / 2:
            # the phase k y / L of node y = b (j + t) / P is k (j + t) / (2P):
            # its integer part k j is reduced mod 2P exactly, so the cosine's
            # argument carries only the rounding of k t (with the phase
            # formed from y itself, the rounding of y alone left ~1e-17 of
            # the tables' scale at k = n against 40-digit mpmath)
            kj = (kint[:, None] * j[None, :]) % (2 * panels)
            num = kj[:, :, None].astype(_LD) + k[:, None, None] * t[None, None, :]
            c = np.cos(two_pi * num.reshape(n + 1, -1) / _LD(2 * panels))
        else:
            c = np.cos((two_pi / Ll) * np.outer(k, y))
        J0[s] = (2 * (c @ g)).astype(np.float64)
        J2[s] = (2 * (c @ (y * y * g))).astype(np.float64)

    # the Gaussian-sum terms are independent: one row per thread (numpy
    # releases the interpreter lock inside these array operations)
    with _futures.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(row, range(alpha.size)))
    return J0, J2


def _per_axis(t):
    """Three per-axis items from one shared item or a sequence of three."""
    if isinstance(t, (list, tuple)):
        assert len(t) == 3
        return list(t)
    return [t, t, t]


def spectrum_octant(omega, J0, J2):
    """``Vhat[a,b,c] = sum_s w_s (J2_s(a) J0_s(b) J0_s(c) + J0_s(a) J2_s(b)
    J0_s(c) + J0_s(a) J0_s(b) J2_s(c))`` for a, b, c in 0..n (eq. Gten_sep),
    the tables of a from axis 1, of b from axis 2, of c from axis 3 (J0, J2:
    one table pair shared by the axes, or a sequence of three).

    Vhat is even in every wavenumber component, so this octant of
    non-negative |k_p| holds the whole padded-grid spectrum.  Each of the
    three terms is a sum over s of products of three 1D factors: written as
    one matrix product (library routine) of the (a, b) products and the c
    factor.
    """
    (x0, y0, z0), (x2, y2, z2) = _per_axis(J0), _per_axis(J2)
    na, nb, nc = x0.shape[1], y0.shape[1], z0.shape[1]
    om = np.asarray(omega, dtype=np.float64)
    V = np.zeros((na * nb, nc))
    # each of the three sums over s is one matrix product: the (a, b) rows
    # w_s f_s(a) g_s(b) times the s-by-c table of the third factor
    for fa, fb, fc in ((x2, y0, z0), (x0, y2, z0), (x0, y0, z2)):
        ab = (om[:, None, None] * fa[:, :, None] * fb[:, None, :]).reshape(len(om), na * nb)
        V += ab.T @ fc
    return V.reshape(na, nb, nc)


def multiplier_octant(V, n, L):
    """``m[a,b,c] = -(2 pi)^2 (a^2/L_1^2 + b^2/L_2^2 + c^2/L_3^2) Vhat[a,b,c]
    / (8 n_1 n_2 n_3)`` (n: one count or one per axis; L: one period, or one
    per axis).

    The spectral Laplacian ``-(2 pi/L)^2 |k|^2`` of eq. convtheorem (per axis
    on a rectangular box) times the kernel spectrum, with the 1/(2n)^3 of
    the forward DFT (the trapezoid approximation of the Fourier
    coefficients) folded in.
    """
    L1, L2, L3 = [float(v) for v in _per_axis(L)]
    n1, n2, n3 = counts(n)
    a = np.arange(n1 + 1, dtype=np.float64)[:, None, None]
    b = np.arange(n2 + 1, dtype=np.float64)[None, :, None]
    c = np.arange(n3 + 1, dtype=np.float64)[None, None, :]
    w = (2.0 * math.pi / L1) ** 2 * a ** 2 + (2.0 * math.pi / L2) ** 2 * b ** 2 + (2.0 * math.pi / L3) ** 2 * c ** 2
    return -w * V / float(8 * n1 * n2 * n3)


class Setup:
    """Everything Algorithm 1 precomputes for one (n, h, R, eps, delta); h is
    one spacing or one per axis (rectangular box).  The spectrum octant and
    the multiplier are built on first use."""

    def __init__(self, n, h, R, eps=None, delta=None):
        d_eps, d_delta = default_eps_delta(n, h)
        self.n, self.h, self.R = n, h, R
        self.ns = counts(n)
        self.hs = spacings(h)
        self.Ls = tuple(2.0 * m * v for m, v in zip(self.ns, self.hs))
        self.cubic = len(set(self.hs)) == 1 and len(set(self.ns)) == 1
        self.L = self.Ls[0] if self.cubic else self.Ls
        self.eps = d_eps if eps is None else eps
        self.delta = d_delta if delta is None else delta
        self.omega, self.alpha = gs_weights(R, self.eps, self.delta)
        tables = {}
        for m, Lp in zip(self.ns, self.Ls):
            if (m, Lp) not in tables:
                tables[(m, Lp)] = tables_1d(self.alpha, m, Lp)
        self.J0s = [tables[key][0] for key in zip(self.ns, self.Ls)]
        self.J2s = [tables[key][1] for key in zip(self.ns, self.Ls)]
        self.J0, self.J2 = self.J0s[0], self.J2s[0]
        self._V = None
        self._m = None

    @property
    def V(self):
        if self._V is None:
            self._V = spectrum_octant(self.omega, self.J0s, self.J2s)
        return self._V

    @property
    def m(self):
        if self._m is None:
            self._m = multiplier_octant(self.V, self.ns, self.Ls)
        return self._m

    def full_multiplier(self):
        """The multiplier on the whole padded grid (2 n_p per axis), DFT index
        order."""
        ax = []
        for m in self.ns:
            idx = np.arange(2 * m)
            ax.append(np.minimum(idx, 2 * m - idx))    # |k| for k = idx or idx - 2n
        return self.m[np.ix_(*ax)]


def setup(n, h, R, eps=None, delta=None) -> Setup:
    return Setup(n, h, R, eps, delta)


# --------------------------------------------------------------------------
# The oracle's own FFT: recursive decimation in time, radix 2 and 3,
# full complex, no pruning.
# --------------------------------------------------------------------------


def fft_naive(x, sign: int = -1):
    """Unnormalised DFT ``X[k] = sum_j x[j] exp(sign 2 pi i j k / N)`` along the
    last axis, for N a product of 2s and 3s."""
    x = np.asarray(x, dtype=np.complex128)
    N = x.shape[-1]
    if N == 1:
        return x.copy()
    if N % 2 == 0:
        p = 2
    elif N % 3 == 0:
        p = 3
    else:
        raise ValueError("length %d is not a product of 2s and 3s" % N)
    M = N // p
    subs = [fft_naive(x[..., r::p], sign) for r in range(p)]
    k = np.arange(N)
    out = np.zeros(x.shape[:-1] + (N,), dtype=np.complex128)
    for r in range(p):
        ang = sign * 2.0 * math.pi * ((r * k) % N) / N
        tw = np.cos(ang) + 1j * np.sin(ang)
        out += tw * subs[r][..., k % M]
    return out


def fftn_naive(x, sign: int = -1):
    """fft_naive along every axis of a 3D array."""
    y = np.asarray(x, dtype=np.complex128)
    for ax in range(3):
        y = np.moveaxis(fft_naive(np.moveaxis(y, ax, -1), sign), -1, ax)
    return y


# --------------------------------------------------------------------------
# Algorithm 2: pad, forward FFT, multiply, inverse FFT, crop.
# --------------------------------------------------------------------------


def fftn_c(x, sign: int = -1):
    """The transform of fftn_naive computed by the oracle's C naive FFT
    (``naive_fft.c``: the same recursive radix-2/3 decimation in time, in
    plain C with OpenMP over the independent lines)."""
    from oracle import native
    y = np.array(x, dtype=np.complex128, order="C", copy=True)
    for ax in range(3):
        native.fft_axis_inplace(y, ax, sign)
    return y


def solve_padded(rho, h, R, eps=None, delta=None, su: Setup | None = None, impl: str = "c"):
    """The uncropped result of Algorithm 2 on the padded grid (2 n_p per
    axis; real part).  rho has shape (n_1, n_2, n_3).  impl selects the
    oracle's FFT: "c" (naive_fft.c, fast enough for the full-size grids) or
    "py" (fft_naive, numpy); both are the same unpruned radix-2/3 recursion."""
    rho = np.asarray(rho, dtype=np.float64)
    assert rho.ndim == 3
    if su is None:
        su = setup(_count_of(rho), h, R, eps, delta)
    n1, n2, n3 = rho.shape
    pad = np.zeros((2 * n1, 2 * n2, 2 * n3), dtype=np.complex128)
    pad[:n1, :n2, :n3] = rho                    # zero padding, factor 2
    if impl == "py":
        rhohat = fftn_naive(pad, -1)            # forward DFT (1/(2n)^3 is in m)
        prod = su.full_multiplier() * rhohat    # multiply (eq. convtheorem)
        return fftn_naive(prod, +1).real        # inverse sum, real part
    if impl != "c":
        raise ValueError("impl must be 'c' or 'py'")
    from oracle import native
    for ax in range(3):                         # forward DFT, in place
        native.fft_axis_inplace(pad, ax, -1)
    pad *= su.full_multiplier()                 # multiply (eq. convtheorem)
    for ax in range(3):                         # inverse sum, in place
        native.fft_axis_inplace(pad, ax, +1)
    return pad.real


def solve(rho, h, R, eps=None, delta=None, su: Setup | None = None, impl: str = "c"):
    """u on the original grid (Algorithm 2 with the crop)."""
    n1, n2, n3 = np.asarray(rho).shape
    return np.ascontiguousarray(solve_padded(rho, h, R, eps, delta, su, impl)[:n1, :n2, :n3])


def _count_of(rho):
    """The point count(s) of a density: one int for a cube, else three."""
    s = tuple(np.asarray(rho).shape)
    return s[0] if s[0] == s[1] == s[2] else s


# --------------------------------------------------------------------------
# The same discrete operator without any FFT: a Toeplitz convolution whose
# stencil factors into 1D sums.
# --------------------------------------------------------------------------


def _stencil_factors(su: Setup):
    """1D stencils over offsets d = -(n_p-1)..(n_p-1) for every Gaussian-sum
    term and axis p: ``F[p][f](d) = sum_{k=-n_p}^{n_p-1} f(|k|)
    exp(i pi k d / n_p)`` for f in {J0, J2, k^2 J0, k^2 J2} of axis p's
    tables."""
    out = []
    for n, J0, J2 in zip(su.ns, su.J0s, su.J2s):
        k = np.arange(-n, n)
        d = np.arange(-(n - 1), n)
        ak = np.abs(k)
        # real because f(|k|) is even in k except for the single k = -n
        # term, whose phase exp(-i pi d) = (-1)^d is real
        phase = np.cos(math.pi * np.outer(d, k) / n)
        k2 = (ak * ak).astype(np.float64)
        out.append((J0[:, ak] @ phase.T, J2[:, ak] @ phase.T, (J0[:, ak] * k2) @ phase.T,
                    (J2[:, ak] * k2) @ phase.T))
    return out


def _separable_terms(su: Setup):
    """Yield (s, coef, (t1, t2, t3)) for the stencil
    ``c_d = sum coef * F[0]_t1(d1) F[1]_t2(d2) F[2]_t3(d3)``: the product of
    ``-(2 pi)^2/(8 n_1 n_2 n_3) (k1^2/L_1^2 + k2^2/L_2^2 + k3^2/L_3^2)`` with
    the three rank-one terms of eq. Gten_sep, expanded into nine separable
    terms per Gaussian-sum term.  Factor types: 0 = J0, 1 = J2, 2 = k^2 J0,
    3 = k^2 J2."""
    n1, n2, n3 = su.ns
    C = [-((2.0 * math.pi / Lp) ** 2) / float(8 * n1 * n2 * n3) for Lp in su.Ls]
    for s in range(len(su.omega)):
        for q in range(3):            # which axis carries J2
            for p2 in range(3):       # which axis carries the k^2 factor
                ts = tuple((2 if p == p2 else 0) + (1 if p == q else 0) for p in range(3))
                yield s, C[p2] * su.omega[s], ts


def direct_operator(rho, h, R, eps=None, delta=None, su: Setup | None = None):
    """u_j = sum_m c_{j-m} rho_m over the whole grid, no FFT.  Cost
    O(R n^4) through the separable stencil; intended for n <= 32."""
    rho = np.asarray(rho, dtype=np.float64)
    if su is None:
        su = setup(_count_of(rho), h, R, eps, delta)
    F = _stencil_factors(su)
    off = []
    for n in rho.shape:
        j = np.arange(n)
        off.append((j[:, None] - j[None, :]) + (n - 1))     # index of d = j - m
    u = np.zeros_like(rho)
    for s, coef, (t1, t2, t3) in _separable_terms(su):
        T1, T2, T3 = F[0][t1][s][off[0]], F[1][t2][s][off[1]], F[2][t3][s][off[2]]
        t = np.tensordot(rho, T3, axes=([2], [1]))          # (m1, m2, j3)
        t = np.tensordot(t, T2, axes=([1], [1]))             # (m1, j3, j2)
        t = np.tensordot(t, T1, axes=([0], [1]))             # (j3, j2, j1)
        u += coef * np.transpose(t, (2, 1, 0))
    return u


def direct_points(rho, points, h, R, eps=None, delta=None, su: Setup | None = None):
    """u at selected grid indices ``points`` (array of shape (P, 3)) by the
    same FFT-free Toeplitz sum; usable at any n."""
    rho = np.asarray(rho, dtype=np.float64)
    if su is None:
        su = setup(_count_of(rho), h, R, eps, delta)
    n1, n2, n3 = rho.shape
    F = _stencil_factors(su)
    pts = np.asarray(points, dtype=np.int64).reshape(-1, 3)
    j3s, inv3 = np.unique(pts[:, 2], return_inverse=True)
    out = np.zeros(pts.shape[0])
    rho2 = rho.reshape(n1 * n2, n3)
    d3 = (j3s[:, None] - np.arange(n3)[None, :]) + (n3 - 1)
    d1 = (pts[:, 0][:, None] - np.arange(n1)[None, :]) + (n1 - 1)
    d2 = (pts[:, 1][:, None] - np.arange(n2)[None, :]) + (n2 - 1)
    cache = {}
    for s, coef, (t1, t2, t3) in _separable_terms(su):
        key = (s, t3)
        if key not in cache:
            cache.clear() if len(cache) > 8 else None
            cache[key] = (rho2 @ F[2][t3][s][d3].T).reshape(n1, n2, -1)[:, :, inv3]
        tp = cache[key]                                        # (m1, m2, P)
        out += coef * np.einsum("pa,pb,abp->p", F[0][t1][s][d1], F[1][t2][s][d2], tp,
                                optimize=True)
    return out
