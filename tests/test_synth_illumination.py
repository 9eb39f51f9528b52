"""Pins of the alternative light-sheet illuminations (Bessel beam, Bessel
lattice) of the input generators.

* a thin-annulus Bessel beam has the J0(k_r r)^2 core near the axis;
* the spectra live on the annulus only;
* a square lattice whose four wavevectors fall on grid points is the closed
  form |2 cos(k x) + 2 cos(k y)|^2 and keeps its intensity exactly along a
  clear-medium march (all four modes share one kz);
* the spots of a hexagonal lattice sit at the six expected azimuths.
"""
import numpy as np
from scipy.special import j0

import oracle
import synth

N, DX, LAM, N0 = 256, 0.2, 0.5, 1.33


def test_bessel_core_is_j0_squared():
    u = synth.bessel_field(N, N, DX, LAM, N0, 0.55, 0.50).astype(complex)
    inten = np.abs(u) ** 2
    kr = 2 * np.pi / LAM * 0.525
    r = np.arange(9) * DX
    for line in (inten[N // 2, N // 2:N // 2 + 9], inten[N // 2:N // 2 + 9, N // 2]):
        assert np.abs(line / line[0] - j0(kr * r) ** 2).max() <= 0.01
    assert abs(np.linalg.norm(u) - 1) <= 1e-6


def test_spectra_live_on_the_annulus():
    k0 = 2 * np.pi / LAM
    kx = 2 * np.pi * np.fft.fftfreq(N, d=DX)
    kt = np.hypot(kx[None, :], kx[:, None])
    for spec in (synth.bessel_spectrum(N, N, DX, LAM, N0, 0.5, 0.4),
                 synth.lattice_spectrum(N, N, DX, LAM, N0, 0.5, 0.4, 6, (0.1, 0.02))):
        on = np.abs(spec) > 0
        assert on.any() and kt[on].min() >= k0 * 0.4 - 1e-9 and kt[on].max() <= k0 * 0.5 + 1e-9


def test_grid_exact_square_lattice():
    p = 20
    na_r = p * LAM / (N * DX)
    spec = synth.lattice_spectrum(N, N, DX, LAM, N0, na_r + 0.02, na_r - 0.02, 4, 1e-4, 0.0)
    assert np.count_nonzero(np.abs(spec) > 1e-300) == 4
    u = np.fft.ifft2(spec)
    y, x = np.mgrid[0:N, 0:N]
    k = 2 * np.pi * p / (N * DX)
    ref = np.abs(np.cos(k * x * DX) + np.cos(k * y * DX)) ** 2 * (2 / N ** 2) ** 2
    inten = np.abs(u) ** 2
    assert np.abs(inten - ref).max() <= 1e-12 * ref.max()
    out, _ = oracle.bpm_forward(u, np.zeros((40, N, N)), DX, 0.2, LAM, N0, intensity=False)
    assert np.abs(np.abs(out) ** 2 - inten).max() <= 1e-12 * inten.max()


def test_hexagonal_lattice_spots():
    k0 = 2 * np.pi / LAM
    spec = np.abs(synth.lattice_spectrum(N, N, DX, LAM, N0, 0.5, 0.4, 6, 0.01, 0.3))
    kx = 2 * np.pi * np.fft.fftfreq(N, d=DX)
    dk = kx[1]
    for m in range(6):
        ph = 0.3 + 2 * np.pi * m / 6
        kxm, kym = k0 * 0.45 * np.cos(ph), k0 * 0.45 * np.sin(ph)
        near = (np.abs(kx[None, :] - kxm) <= 2 * dk) & (np.abs(kx[:, None] - kym) <= 2 * dk)
        iy, ix = np.unravel_index(np.argmax(np.where(near, spec, 0)), spec.shape)
        assert abs(kx[ix] - kxm) <= dk and abs(kx[iy] - kym) <= dk and spec[iy, ix] > 0.5
