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
