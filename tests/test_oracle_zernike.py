"""Pins of the aberration-map oracle (oracle/zernike.py).

* Noll ordering of the first indices and orthonormality of Z_1 .. Z_28 over
  the unit disc (Gauss-Legendre x uniform-angle quadrature);
* a pupil with a pure lateral-shift ramp exp(-i kx s) is fitted exactly by
  tilt: c_2 = -k0 NA s_x / 2, c_3 = -k0 NA s_y / 2, nothing else (also for
  shifts whose ramp wraps several times across the pupil);
* astigmatism a rho^2 cos 2 theta and b rho^2 sin 2 theta: c_6 = a / sqrt 6,
  c_5 = b / sqrt 6;
* a pure defocus exp(i (kz - k) dz) has only terms that the square sampling
  grid's symmetry allows (m = 0, and tiny cos 4 theta), with the sign of dz;
* end to end: a clear-medium march of a source displaced by s pixels, read
  with the window centred on the undisplaced pixel, gives c_2 = -k0 NA s dx / 2
  within the window's truncation, and a centred source gives no aberration.
"""
import math

import numpy as np

import oracle
import synth
from oracle import zernike as zo

LAM, N0, NA, DX = 0.5, 1.33, 0.6, 0.2
K0 = 2 * np.pi / LAM


def test_noll_order():
    got = [zo.noll_nm(j) for j in range(1, 12)]
    assert got == [(0, 0), (1, 1), (1, -1), (2, 0), (2, -2), (2, 2), (3, -1), (3, 1), (3, -3),
                   (3, 3), (4, 0)]


def test_orthonormal_on_the_unit_disc():
    x, w = np.polynomial.legendre.leggauss(40)
    r = 0.5 * (x + 1)
    wr = 0.5 * w
    th = 2 * np.pi * np.arange(64) / 64
    R, TH = np.meshgrid(r, th, indexing="ij")
    W = (wr * r)[:, None] * (2 * np.pi / 64)
    Z = np.stack([zo.zernike(j, R, TH) for j in range(1, 29)])
    G = np.einsum("iab,jab,ab->ij", Z, Z, W) / np.pi
    assert np.abs(G - np.eye(28)).max() <= 1e-10


def pupil_of(phase_fn, crop=32):
    """Unit-amplitude pupil field with the window-centre convention."""
    mask, rho, theta = zo.disc(crop, DX, LAM, NA)
    sign = (-1.0) ** (np.arange(crop)[:, None] + np.arange(crop)[None, :])
    X = np.where(mask, np.exp(1j * phase_fn(rho, theta)), 0.0) * sign
    return X[None]


def test_tilt_is_fitted_exactly():
    for sx, sy in [(0.2, 0.0), (-0.1, 0.3), (0.9, -0.7)]:        # up to ~7 rad at the rim
        X = pupil_of(lambda r, t: -K0 * NA * r * (np.cos(t) * sx + np.sin(t) * sy))
        c, rms = zo.zernike_fit(X, DX, LAM, NA, 15)
        ref = np.zeros(15)
        ref[1], ref[2] = -K0 * NA * sx / 2, -K0 * NA * sy / 2
        assert np.abs(c[0] - ref).max() <= 1e-10 and rms[0] <= 1e-10


def test_astigmatism_is_fitted_exactly():
    a, b = 0.8, -0.5
    X = pupil_of(lambda r, t: a * r * r * np.cos(2 * t) + b * r * r * np.sin(2 * t))
    c, _ = zo.zernike_fit(X, DX, LAM, NA, 21)
    ref = np.zeros(21)
    ref[5], ref[4] = a / math.sqrt(6), b / math.sqrt(6)
    assert np.abs(c[0] - ref).max() <= 1e-10


def test_defocus_is_rotationally_symmetric():
    k = N0 * K0
    for dz in (0.5, -0.8):
        X = pupil_of(lambda r, t: (np.sqrt(np.maximum(k * k - (K0 * NA * r) ** 2, 0)) - k) * dz)
        c, _ = zo.zernike_fit(X, DX, LAM, NA, 28)
        # the square sampling grid keeps only the symmetry of the square:
        # cos(4 theta) terms may appear, nothing else that depends on theta
        sym = [zo.noll_nm(j)[1] in (0, 4) for j in range(1, 29)]
        assert np.abs(c[0][~np.array(sym)]).max() <= 1e-10
        assert np.abs(c[0][np.array([zo.noll_nm(j)[1] == 4 for j in range(1, 29)])]).max() <= 1e-5
        assert np.sign(c[0][3]) == -np.sign(dz) and abs(c[0][3]) > 0.1


def test_clear_medium_march_gives_the_source_tilt():
    n, steps, crop = 128, 10, 32
    src = np.array([[40, 40], [40, 104], [104, 40], [104, 104]])
    shift = np.array([0, 1, 2, -1])
    placed = src + np.stack([np.zeros(4, int), shift], 1)
    u0 = synth.multiplexed_field(n, n, DX, LAM, N0, NA, 0.0, placed)
    exit_, _ = oracle.bpm_forward(u0, np.zeros((steps, n, n)), DX, 0.2, LAM, N0,
                                  intensity=False)
    X = zo.pupil_fields(exit_, DX, 0.2, LAM, N0, NA, steps, src, crop)
    c, rms = zo.zernike_fit(X, DX, LAM, NA, 15)
    # four sources 64 pixels apart: the window's truncation and the
    # neighbours' light leave ~1e-2 rad
    for s in range(4):
        ref = -K0 * NA * shift[s] * DX / 2
        assert abs(c[s][1] - ref) <= 0.01 * abs(ref) + 0.01
        assert np.abs(np.delete(c[s], [0, 1])).max() <= 2e-2 and rms[s] <= 0.03
    # one source, a 64-pixel window: 2e-3 rad
    u0 = synth.multiplexed_field(n, n, DX, LAM, N0, NA, 0.0, [[64, 65]])
    exit_, _ = oracle.bpm_forward(u0, np.zeros((steps, n, n)), DX, 0.2, LAM, N0,
                                  intensity=False)
    c, _ = zo.zernike_fit(zo.pupil_fields(exit_, DX, 0.2, LAM, N0, NA, steps, [[64, 64]], 64),
                          DX, LAM, NA, 15)
    assert abs(c[0][1] + K0 * NA * DX / 2) <= 2e-3 and np.abs(np.delete(c[0], 1)).max() <= 2e-3
