"""FP64 oracle of the sample-induced aberration maps (main-text paragraph on
the light-sheet simulation: the extraction of sample-induced aberrations as
spatially resolved Zernike maps).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``.

What is computed (numpy, from the definitions):

* pupil fields -- the exit field of a multiplexed march that started at the
  source plane ``back`` slices earlier is brought back to that plane through
  the detection pupil P (NA, integer test as for the PSF readout),
  E0 = IDFT2(DFT2(u) P exp(-i kz back dz)); each source's C x C window
  (source at window index (C/2, C/2)) is transformed,
  X_s(l, m) = sum_{y,x} E0(sy - C/2 + y, sx - C/2 + x) exp(-2 pi i (l y + m x) / C).
* Zernike fit -- on the pupil disc D = {l'^2 + m'^2 <= (NA C dx / lambda)^2}
  (signed frequency indices), rho = |k| / (k0 NA), theta = atan2(ky, kx):
  Y = X (-1)^(l + m) (the window-centre ramp removed); a tilt estimate
  t_x = arg sum Y(l, m+1) conj Y(l, m), t_y likewise, and a piston p0 give
  the reference T = t_x m' + t_y l' + p0; the wavefront is
  W = wrap(arg Y - T) + T; the coefficients of the Noll-normalised Zernike
  polynomials Z_1 .. Z_J are the least-squares fit c = P W, P = (Z^T Z)^-1 Z^T
  over D, followed by two passes c += P wrap(W - Z c) (which remove the effect
  of isolated 2 pi branch jumps of W); rms = sqrt(mean_D wrap(W - Z c)^2).
* Zernike polynomials (Noll 1976): j -> (n, m); Z_j = sqrt(n + 1) R_n^0 for
  m = 0, sqrt(2 (n + 1)) R_n^m cos(m theta) for even j and ... sin(m theta)
  for odd j, R_n^m the radial polynomial's factorial sum.

Parity status (tests/test_oracle_zernike.py): orthonormality on the unit disc
by quadrature; exact recovery of a tilt (c_2 = -k0 NA dx_shift / 2), of
astigmatism and of wrapped tilts; only m = 0 terms for a pure defocus; a
clear-medium march of a displaced source gives its tilt.
"""
from __future__ import annotations

import math

import numpy as np


def noll_nm(j: int):
    """(n, m) of Noll index j >= 1; m < 0 marks the sine term (odd j)."""
    if j < 1:
        raise ValueError("Noll indices start at 1")
    n = int((math.isqrt(8 * j - 7) - 1) // 2)
    k = j - n * (n + 1) // 2 - 1
    m = n % 2 + 2 * ((k + 1 - n % 2) // 2)
    if m != 0 and j % 2 == 1:
        m = -m
    return n, m


def radial(n: int, m: int, rho):
    m = abs(m)
    out = np.zeros_like(np.asarray(rho, float))
    for s in range((n - m) // 2 + 1):
        c = ((-1) ** s * math.factorial(n - s)
             / (math.factorial(s) * math.factorial((n + m) // 2 - s)
                * math.factorial((n - m) // 2 - s)))
        out = out + c * np.asarray(rho, float) ** (n - 2 * s)
    return out


def zernike(j: int, rho, theta):
    """Noll-normalised Z_j (unit mean square over the unit disc)."""
    n, m = noll_nm(j)
    r = radial(n, m, rho)
    if m == 0:
        return math.sqrt(n + 1) * r
    ang = np.cos(m * np.asarray(theta)) if m > 0 else np.sin(-m * np.asarray(theta))
    return math.sqrt(2 * (n + 1)) * r * ang


def wrap(p):
    return p - 2.0 * np.pi * np.floor((p + np.pi) / (2.0 * np.pi))


def _signed(n):
    i = np.arange(n)
    return np.where(i < n // 2, i, i - n)


def refocused_plane(exit_field, dx, dz, wavelength, n0, na, back_steps):
    """E0 = IDFT2(DFT2(u) P exp(-i kz back dz))."""
    u = np.asarray(exit_field, complex)
    ny, nx = u.shape
    ms, ls = _signed(nx)[None, :], _signed(ny)[:, None]
    kx = 2 * np.pi * ms / (nx * dx)
    ky = 2 * np.pi * ls / (ny * dx)
    k = 2 * np.pi * n0 / wavelength
    kz = np.sqrt(np.maximum(k * k - kx ** 2 - ky ** 2, 0.0))
    thr = (nx * ny * na * dx / wavelength) ** 2
    pupil = (ms * ny) ** 2 + (ls * nx) ** 2 <= thr
    S = np.fft.fft2(u) * pupil * np.exp(-1j * kz * back_steps * dz)
    return np.fft.ifft2(S)


def pupil_fields(exit_field, dx, dz, wavelength, n0, na, back_steps, sources, crop):
    """X [n_src][crop][crop]: the DFT of each source's window of E0."""
    E = refocused_plane(exit_field, dx, dz, wavelength, n0, na, back_steps)
    ny, nx = E.shape
    out = []
    for sy, sx in np.asarray(sources, int).reshape(-1, 2):
        ys = (np.arange(crop) + sy - crop // 2) % ny
        xs = (np.arange(crop) + sx - crop // 2) % nx
        out.append(np.fft.fft2(E[np.ix_(ys, xs)]))
    return np.array(out).reshape(-1, crop, crop)


def disc(crop, dx, wavelength, na):
    """(mask, rho, theta) on the crop's DFT grid."""
    m = _signed(crop)[None, :].astype(float)
    l = _signed(crop)[:, None].astype(float)
    R = na * crop * dx / wavelength
    mask = np.broadcast_to(l ** 2 + m ** 2 <= R * R, (crop, crop))
    rho = np.sqrt(l ** 2 + m ** 2) / R
    theta = np.arctan2(np.broadcast_to(l, (crop, crop)), np.broadcast_to(m, (crop, crop)))
    return mask, rho, theta


def zernike_fit(pupil, dx, wavelength, na, n_modes, passes=2):
    """(coefficients [n_src][n_modes], rms [n_src]) of the pupil fields."""
    X = np.asarray(pupil, complex)
    n_src, crop, _ = X.shape
    mask, rho, theta = disc(crop, dx, wavelength, na)
    Z = np.stack([zernike(j, rho[mask], theta[mask]) for j in range(1, n_modes + 1)], axis=1)
    P = np.linalg.solve(Z.T @ Z, Z.T)
    ls, ms = _signed(crop)[:, None], _signed(crop)[None, :]
    sign = (-1.0) ** (np.arange(crop)[:, None] + np.arange(crop)[None, :])
    pair_x = mask & np.roll(mask, -1, axis=1)
    pair_y = mask & np.roll(mask, -1, axis=0)
    coeffs, rms = [], []
    for s in range(n_src):
        Y = X[s] * sign
        tx = np.angle(np.sum((np.roll(Y, -1, axis=1) * np.conj(Y))[pair_x]))
        ty = np.angle(np.sum((np.roll(Y, -1, axis=0) * np.conj(Y))[pair_y]))
        ramp = np.broadcast_to(tx * ms + ty * ls, (crop, crop))
        p0 = np.angle(np.sum((Y * np.exp(-1j * ramp))[mask]))
        T = (ramp + p0)[mask]
        W = wrap(np.angle(Y[mask]) - T) + T
        c = P @ W
        for _ in range(passes):
            c = c + P @ wrap(W - Z @ c)
        coeffs.append(c)
        rms.append(math.sqrt(np.mean(wrap(W - Z @ c) ** 2)))
    return np.array(coeffs), np.array(rms)
