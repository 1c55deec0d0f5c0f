"""Pins for the oracle's own FFT against numpy's (a library routine used here
only as a comparator) and against the DFT definition."""
import math

import numpy as np
import pytest

from oracle import psp_oracle as O

LENGTHS = [1, 2, 3, 4, 6, 8, 9, 12, 16, 18, 24, 27, 32, 48, 64, 96, 128, 192, 256]


@pytest.mark.parametrize("N", LENGTHS)
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft_matches_numpy(N, sign):
    rng = np.random.default_rng(N)
    x = rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N))
    got = O.fft_naive(x, sign)
    want = np.fft.fft(x, axis=-1) if sign < 0 else np.fft.ifft(x, axis=-1) * N
    assert np.max(np.abs(got - want)) <= 1e-14 * max(1.0, np.max(np.abs(want))) * math.log2(2 * N)


@pytest.mark.parametrize("N", [5, 10, 7])
def test_fft_rejects_other_primes(N):
    with pytest.raises(ValueError):
        O.fft_naive(np.ones(N), -1)


def test_fft_definition_small():
    # brute-force DFT sum for a length with both radices
    N = 12
    rng = np.random.default_rng(1)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    j = np.arange(N)
    want = np.array([np.sum(x * np.exp(-2j * math.pi * j * k / N)) for k in range(N)])
    assert np.allclose(O.fft_naive(x, -1), want, atol=1e-13, rtol=0)


def test_roundtrip_and_fftn():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((6, 8, 12))
    X = O.fftn_naive(x, -1)
    assert np.allclose(X, np.fft.fftn(x), atol=1e-12, rtol=0)
    back = O.fftn_naive(X, +1) / x.size
    assert np.max(np.abs(back - x)) < 1e-14


# ---- the same recursion in plain C (oracle/naive_fft.c), which the oracle's
# solve uses by default: pinned to the library FFT and the DFT definition on
# every axis, and to the numpy recursion on whole solves
C_LENGTHS = [1, 2, 3, 4, 6, 8, 9, 12, 18, 27, 36, 64, 72, 81, 96, 108, 144, 162, 216, 288, 324, 384, 432, 512,
             576, 648, 768]


@pytest.mark.parametrize("N", C_LENGTHS)
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_c_fft_matches_numpy_on_every_axis(N, axis):
    from oracle import native
    rng = np.random.default_rng(N + 7 * axis)
    shape = [3, 2, 2]
    shape[axis] = N
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    for sign in (-1, 1):
        y = np.ascontiguousarray(x)
        y = y.copy()
        native.fft_axis_inplace(y, axis, sign)
        want = np.fft.fft(x, axis=axis) if sign < 0 else np.fft.ifft(x, axis=axis) * N
        assert np.max(np.abs(y - want)) <= 1e-14 * max(1.0, np.max(np.abs(want))) * math.log2(2 * N)


def test_c_fft_definition_and_rejects():
    from oracle import native
    N = 18
    rng = np.random.default_rng(5)
    x = (rng.standard_normal(N) + 1j * rng.standard_normal(N)).reshape(1, 1, N)
    j = np.arange(N)
    want = np.array([np.sum(x[0, 0] * np.exp(2j * math.pi * j * k / N)) for k in range(N)])
    y = x.copy()
    native.fft_axis_inplace(y, 2, +1)
    assert np.allclose(y[0, 0], want, atol=1e-13, rtol=0)
    with pytest.raises(ValueError):
        native.fft_axis_inplace(np.ones((1, 1, 10), complex), 2, -1)


@pytest.mark.parametrize("n", [6, 9, 16])
def test_c_solve_equals_numpy_recursion_and_toeplitz(n):
    rng = np.random.default_rng(60 + n)
    rho = rng.standard_normal((n, n, n))
    h = 2.0 / n
    su = O.setup(n, h, 12)
    uc = O.solve(rho, h, 12, su=su, impl="c")
    up = O.solve(rho, h, 12, su=su, impl="py")
    ud = O.direct_operator(rho, h, 12, su=su)
    scale = np.max(np.abs(ud))
    assert np.max(np.abs(uc - up)) <= 1e-14 * scale
    assert np.max(np.abs(uc - ud)) <= 1e-14 * scale
