"""Pins of the oracle's radix-2 FFT against the plain O(N^2) definition.

The definition X[k] = sum_n x[n] exp(sign 2 pi i n k / N) is written out here
in pure Python (cmath, lists), independently of the C code, on tiny sizes.
"""
import cmath
import random

import numpy as np
import pytest

import oracle


def dft_bruteforce(x, sign):
    n = len(x)
    return [sum(x[t] * cmath.exp(sign * 2j * cmath.pi * t * k / n) for t in range(n))
            for k in range(n)]


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft1d_matches_definition(n, sign):
    r = random.Random(n * 7 + sign)
    x = [complex(r.gauss(0, 1), r.gauss(0, 1)) for _ in range(n)]
    ref = dft_bruteforce(x, sign)
    got = oracle.fft1d(np.array(x), sign)
    err = max(abs(a - b) for a, b in zip(got, ref))
    assert err <= 1e-12 * max(1.0, n)


def test_fft2d_matches_definition():
    r = random.Random(5)
    ny, nx = 4, 8
    x = [[complex(r.gauss(0, 1), r.gauss(0, 1)) for _ in range(nx)] for _ in range(ny)]
    ref = [[sum(x[b][a] * cmath.exp(-2j * cmath.pi * (a * m / nx + b * l / ny))
                for b in range(ny) for a in range(nx)) for m in range(nx)] for l in range(ny)]
    got = oracle.fft2d(np.array(x), -1)
    assert np.abs(got - np.array(ref)).max() <= 1e-12


def test_fft_round_trip():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((64, 256)) + 1j * rng.standard_normal((64, 256))
    y = oracle.fft2d(oracle.fft2d(x, -1), +1) / x.size
    assert np.abs(y - x).max() <= 1e-13


def test_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        oracle.fft1d(np.zeros(12), -1)
