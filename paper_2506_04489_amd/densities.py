"""Seeded synthetic densities on uniform grids (inputs only).

This module builds the right-hand sides rho that the solver and the CPU
checker both consume.  It holds none of the solver's arithmetic: no Green's
function, no Gaussian-sum fit, no transform.  Every function works on the
host with numpy and, through ``xp=torch`` plus a ``device``, on the GPU.

Grid convention: ``x_j = x0 + j*h`` for ``j = 0..n-1`` along each axis, the
array is C-ordered ``rho[i1, i2, i3]`` with ``i3`` contiguous.

Density families (the paper's benchmark families, Section 3):
  * isotropic Gaussian ``exp(-|x-c|^2 / a^2)``;
  * normalised Gaussian ``(2 pi)^{-3/2} sigma^{-3} exp(-|x-c|^2/(2 sigma^2))``
    (the paper's Gaussian source, Section 3.2);
  * separable oscillatory ``exp(-|x|^2/a^2) sin(w x1) cos(w x2) sin(w x3)``;
  * C-infinity bump ``exp(-1/(1 - r^2/R^2))`` for ``r < R``;
  * mixtures of 1-4 Gaussians with random centres, widths and amplitudes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def _ns(xp):
    """Return (module, is_torch) for an array namespace argument."""
    if xp is None or xp is np:
        return np, False
    return xp, True


def axis_coords(n: int, h: float, x0: float, xp=None, dtype=None, device=None):
    """1D coordinates ``x0 + j*h``, j = 0..n-1, as float64 (or ``dtype``)."""
    mod, is_torch = _ns(xp)
    if is_torch:
        dt = dtype if dtype is not None else mod.float64
        return x0 + h * mod.arange(n, dtype=dt, device=device)
    dt = dtype if dtype is not None else np.float64
    return (x0 + h * np.arange(n, dtype=np.float64)).astype(dt)


def _grid3(n, h, x0, xp, device, centre=(0.0, 0.0, 0.0)):
    if not isinstance(n, (tuple, list)):
        n = (n, n, n)
    if not isinstance(h, (tuple, list)):
        h = (h, h, h)
    if not isinstance(x0, (tuple, list)):
        x0 = (x0, x0, x0)
    xs = [axis_coords(n[p], h[p], x0[p], xp=xp, device=device) - centre[p] for p in range(3)]
    return xs[0][:, None, None], xs[1][None, :, None], xs[2][None, None, :]


def gaussian(n, h, x0, a, centre=(0.0, 0.0, 0.0), xp=None, device=None):
    """``exp(-|x - c|^2 / a^2)`` sampled on the grid."""
    mod, _ = _ns(xp)
    X, Y, Z = _grid3(n, h, x0, xp, device, centre)
    return mod.exp(-(X * X + Y * Y + Z * Z) / (a * a))


def normalised_gaussian(n, h, x0, sigma, centre=(0.0, 0.0, 0.0), xp=None, device=None):
    """The paper's Gaussian source: unit mass, standard deviation ``sigma``."""
    mod, _ = _ns(xp)
    X, Y, Z = _grid3(n, h, x0, xp, device, centre)
    c = 1.0 / ((2.0 * math.pi) ** 1.5 * sigma ** 3)
    return c * mod.exp(-(X * X + Y * Y + Z * Z) / (2.0 * sigma * sigma))


def oscillatory(n, h, x0, a=0.2, omega=20.0, centre=(0.0, 0.0, 0.0), xp=None, device=None):
    """``exp(-|x|^2/a^2) sin(w x1) cos(w x2) sin(w x3)``."""
    mod, _ = _ns(xp)
    X, Y, Z = _grid3(n, h, x0, xp, device, centre)
    return (mod.exp(-(X * X + Y * Y + Z * Z) / (a * a))
            * mod.sin(omega * X) * mod.cos(omega * Y) * mod.sin(omega * Z))


def bump(n, h, x0, radius=0.6, centre=(0.0, 0.0, 0.0), xp=None, device=None):
    """C-infinity bump ``exp(-1/(1 - r^2/R^2))`` inside ``r < R``, zero outside.

    The exponent is guarded so that no division by zero or overflow occurs at
    or outside the support boundary.
    """
    mod, _ = _ns(xp)
    X, Y, Z = _grid3(n, h, x0, xp, device, centre)
    t = (X * X + Y * Y + Z * Z) / (radius * radius)
    inside = t < 1.0
    one_minus = mod.where(inside, 1.0 - t, mod.ones_like(t))
    val = mod.exp(-1.0 / one_minus)
    return mod.where(inside, val, mod.zeros_like(val))


@dataclass
class Mixture:
    """A sum of isotropic Gaussians ``sum_i A_i exp(-|x - c_i|^2 / (2 s_i^2))``."""
    centres: list = field(default_factory=list)
    sigmas: list = field(default_factory=list)
    amps: list = field(default_factory=list)

    def sample(self, n, h, x0, xp=None, device=None):
        mod, _ = _ns(xp)
        out = None
        for c, s, A in zip(self.centres, self.sigmas, self.amps):
            X, Y, Z = _grid3(n, h, x0, xp, device, c)
            g = A * mod.exp(-(X * X + Y * Y + Z * Z) / (2.0 * s * s))
            out = g if out is None else out + g
        return out


def draw_mixture(rng: np.random.Generator) -> Mixture:
    """1-4 Gaussians: centres U[-0.5,0.5]^3, widths U[0.08,0.2], amplitudes N(0,1)."""
    k = int(rng.integers(1, 5))
    centres = [tuple(float(v) for v in rng.uniform(-0.5, 0.5, size=3)) for _ in range(k)]
    sigmas = [float(v) for v in rng.uniform(0.08, 0.2, size=k)]
    amps = [float(v) for v in rng.normal(0.0, 1.0, size=k)]
    return Mixture(centres, sigmas, amps)


# Workload seeds (PCG64 via numpy.random.default_rng).
BATCH_SEED = 2506
SERVE_SEED = 4489
BATCH_SIZES = (32, 48, 64, 96, 128)
SERVE_SIZES = (64, 96, 128, 192, 256, 384)
SERVE_PROBS = (0.25, 0.20, 0.20, 0.15, 0.12, 0.08)


@dataclass
class BatchItem:
    n: int
    h: float
    x0: float
    mixture: Mixture


def batched_workload(count: int = 64, seed: int = BATCH_SEED):
    """The batched workload: ``count`` densities, n ~ U{32,48,64,96,128} on
    the cube [-1,1)^3 with h = 2/n, each a seeded Gaussian mixture."""
    rng = np.random.default_rng(seed)
    items = []
    for _ in range(count):
        n = int(rng.choice(BATCH_SIZES))
        items.append(BatchItem(n=n, h=2.0 / n, x0=-1.0, mixture=draw_mixture(rng)))
    return items


@dataclass
class Request:
    t_arrival: float      # seconds after stream start
    n: int
    h: float
    x0: float
    tier: str             # "f64" or "f32"
    kind: str             # "mixture" or "oscillatory"
    mixture: Mixture | None
    omega: float


def serving_workload(count: int = 2000, rate: float = 100.0, seed: int = SERVE_SEED):
    """The serving stream: Poisson arrivals at ``rate`` req/s, n drawn from
    {64,96,128,192,256,384} with probabilities {.25,.2,.2,.15,.12,.08},
    densities 50/50 mixture or oscillatory (omega ~ U[5,25]), tier 50/50."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for _ in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = int(rng.choice(SERVE_SIZES, p=SERVE_PROBS))
        kind = "mixture" if rng.random() < 0.5 else "oscillatory"
        mix = draw_mixture(rng) if kind == "mixture" else None
        omega = float(rng.uniform(5.0, 25.0))
        tier = "f64" if rng.random() < 0.5 else "f32"
        reqs.append(Request(t, n, 2.0 / n, -1.0, tier, kind, mix, omega))
    return reqs


def request_density(req: Request, xp=None, device=None):
    if req.kind == "mixture":
        return req.mixture.sample(req.n, req.h, req.x0, xp=xp, device=device)
    return oscillatory(req.n, req.h, req.x0, a=0.2, omega=req.omega, xp=xp, device=device)
