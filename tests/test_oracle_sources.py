"""Pins of the oracle's multiplexed point-source field.

* one source at the origin is numpy's inverse FFT of the closed-form
  Gaussian-apodised NA-limited spectrum (a library routine), scaled to unit
  norm, for in-focus and defocused sources;
* a source at p is the origin source circularly shifted by p;
* the field is linear in the per-source weights exp(i phase);
* it agrees with the input generator's comb-convolution construction.
"""
import numpy as np
import pytest

import oracle
import synth

LAM, N0, NA = 0.5, 1.33, 0.6


def closed_form(n, dx, z_d):
    k0 = 2 * np.pi / LAM
    k = N0 * k0
    f = 2 * np.pi * np.fft.fftfreq(n, d=dx)
    kt2 = f[None, :] ** 2 + f[:, None] ** 2
    kmax2 = (k0 * NA) ** 2
    kz = np.sqrt(np.maximum(k * k - kt2, 0.0))
    spec = np.where(kt2 <= kmax2, np.exp(-kt2 / kmax2) * np.exp(-1j * kz * z_d), 0.0)
    u = np.fft.ifft2(spec)
    return u / np.linalg.norm(u)


@pytest.mark.parametrize("n,dx,z_d", [(64, 0.2, 0.0), (32, 0.1, 2.0), (128, 0.2, -1.5)])
def test_single_source_is_the_closed_form(n, dx, z_d):
    u = oracle.point_sources(n, n, dx, LAM, N0, NA, z_d, [(0, 0)])
    ref = closed_form(n, dx, z_d)
    assert np.abs(u - ref).max() <= 1e-12
    assert abs(np.linalg.norm(u) - 1.0) <= 1e-12


def test_shift_and_linearity():
    n = 64
    base = oracle.point_sources(n, n, 0.2, LAM, N0, NA, 1.0, [(0, 0)])
    pos = [(5, 60), (33, 2), (63, 63)]
    ph = [0.4, -2.0, 3.0]
    for p in pos:
        u = oracle.point_sources(n, n, 0.2, LAM, N0, NA, 1.0, [p])
        assert np.abs(u - np.roll(base, p, axis=(0, 1))).max() <= 1e-13
    u = oracle.point_sources(n, n, 0.2, LAM, N0, NA, 1.0, pos, ph)
    ref = sum(np.exp(1j * a) * np.roll(base, p, axis=(0, 1)) for p, a in zip(pos, ph))
    assert np.abs(u - ref).max() <= 1e-13
    assert np.abs(oracle.point_sources(n, n, 0.2, LAM, N0, NA, 1.0, [])).max() == 0.0


def test_matches_the_input_generator():
    n = 128
    gen = np.random.default_rng(5)
    pos = synth.jittered_grid(n, n, 32, 3, gen)
    ph = gen.uniform(0, 2 * np.pi, len(pos))
    u = oracle.point_sources(n, n, 0.2, LAM, N0, NA, 2.0, pos, ph)
    ref = synth.multiplexed_field(n, n, 0.2, LAM, N0, NA, 2.0, pos, ph)
    assert np.abs(u - ref).max() <= 1e-6 * np.abs(ref).max()
