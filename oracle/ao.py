"""FP64 oracle of the adaptive-optics analysis (main-text paragraph on
adaptive optics; Fig. 2c, d).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: imported by the tests
and the benchmark's CPU leg, never by the product package.

What is computed (numpy on top of the FP64 march and adjoint of oracle.c):

* guide-star correction -- a point at the focus x_f is conjugated back to the
  entrance plane by the adjoint march, M^H e_f (for the one-way march this is
  the guide star's field propagated to the sample surface and phase
  conjugated).  With the entrance spectrum U0 = A exp(i phi) exp(-i kz z_f)
  the focus amplitude is u(x_f) = sum_k conj(G_k) U0_k, G = DFT(M^H e_f)/N;
  for fixed |U0| = A it is largest when every mode has the phase of G, so
  phi* = arg G + kz z_f (Cauchy-Schwarz), and I* = (sum_k A_k |G_k|)^2.
* aiming phase -- the same correction for a clear medium, -(kx x_f + ky y_f):
  the uncorrected wavefront that focuses on x_f without the tissue.
* memory effect -- the corrected entrance field shifted by s (the phase
  minus kx s_x + ky s_y) and marched; persistence P(s) = I_s(x_f + s) / I_0(x_f).
* speckle autocorrelation -- the exit intensity I of an incident plane wave
  and its normalised circular autocovariance C(d) = R(d) / R(0),
  R(d) = sum_x (I(x) - <I>)(I(x + d) - <I>), averaged over the x and y lags.
* mean free paths -- depth in scattering mean free paths from the ballistic
  (unscattered) power of an incident unit plane wave, -ln |<u_N>|^2.

Parity status (tests/test_oracle_ao.py): clear medium gives the aiming
phase and P = 1 exactly; the corrected intensity equals (sum A |G|)^2 and
beats random phases; cosine fringes have C(d) = cos(2 pi d / P); one thin
screen gives -ln |<exp(i k0 dz dn)>|^2.
"""
from __future__ import annotations

import numpy as np

from . import bpm_adjoint, bpm_forward


def wavenumbers(nx, ny, dx, wavelength, n0):
    """kx [1][nx], ky [ny][1], kz [ny][nx] on numpy's FFT grid (rad/um)."""
    k = 2.0 * np.pi * n0 / wavelength
    kx = 2.0 * np.pi * np.fft.fftfreq(nx, d=dx)[None, :]
    ky = 2.0 * np.pi * np.fft.fftfreq(ny, d=dx)[:, None]
    return kx, ky, np.sqrt(np.maximum(k * k - kx ** 2 - ky ** 2, 0.0))


def wrap(p):
    """Angle in [-pi, pi)."""
    return p - 2.0 * np.pi * np.floor((p + np.pi) / (2.0 * np.pi))


def pupil_spectrum(amp, phase, dx, wavelength, n0, z_focus):
    """U0 = A exp(i phi) exp(-i kz z_f) (natural DFT order)."""
    ny, nx = np.shape(amp)
    _, _, kz = wavenumbers(nx, ny, dx, wavelength, n0)
    return np.asarray(amp, float) * np.exp(1j * np.asarray(phase, float)) * np.exp(-1j * kz * z_focus)


def exit_field(amp, phase, dn, dx, dz, wavelength, n0, z_focus):
    """Field at the exit plane of the march started from IDFT(U0)."""
    u0 = np.fft.ifft2(pupil_spectrum(amp, phase, dx, wavelength, n0, z_focus))
    out, _ = bpm_forward(u0, dn, dx, dz, wavelength, n0, intensity=False)
    return out


def guide_star_gradient(dn, focus, dx, dz, wavelength, n0):
    """G = DFT(M^H e_f) / N: the spectrum gradient of Re u(x_f) (focus = (y, x))."""
    ny, nx = np.shape(dn)[1:]
    e = np.zeros((ny, nx), complex)
    e[focus[0], focus[1]] = 1.0
    _, gs, _ = bpm_adjoint(np.zeros((ny, nx), complex), dn, dx, dz, wavelength, n0, grad_u_out=e)
    return gs


def guide_star_phase(gs, dx, wavelength, n0, z_focus, shift=(0.0, 0.0)):
    """phi = arg G + kz z_f - kx shift_x - ky shift_y, wrapped to [-pi, pi)."""
    ny, nx = np.shape(gs)
    kx, ky, kz = wavenumbers(nx, ny, dx, wavelength, n0)
    return wrap(np.angle(gs) + kz * z_focus - kx * shift[0] - ky * shift[1])


def aim_phase(nx, ny, dx, wavelength, n0, focus):
    """-(kx x_f + ky y_f): a clear-medium focus on pixel focus = (y, x)."""
    kx, ky, _ = wavenumbers(nx, ny, dx, wavelength, n0)
    return wrap(-(kx * focus[1] * dx + ky * focus[0] * dx))


def optimum_intensity(amp, gs):
    """(sum_k A_k |G_k|)^2: the largest focus intensity over the pupil phase."""
    return float(np.sum(np.asarray(amp, float) * np.abs(gs))) ** 2


def memory_effect(amp, gs, dn, focus, shifts, dx, dz, wavelength, n0, z_focus):
    """P(s) for integer pixel shifts s = (sy, sx): intensity of the shifted
    correction at the shifted focus over the unshifted focus intensity."""
    ny, nx = np.shape(amp)
    base = None
    out = []
    for sy, sx in [(0, 0)] + [tuple(s) for s in shifts]:
        ph = guide_star_phase(gs, dx, wavelength, n0, z_focus, shift=(sx * dx, sy * dx))
        u = exit_field(amp, ph, dn, dx, dz, wavelength, n0, z_focus)
        val = abs(u[(focus[0] + sy) % ny, (focus[1] + sx) % nx]) ** 2
        if base is None:
            base = val
        else:
            out.append(val / base)
    return np.array(out), base


def plane_wave_speckle(dn, dx, dz, wavelength, n0):
    """Exit field of a unit plane wave (normal incidence)."""
    ny, nx = np.shape(dn)[1:]
    out, _ = bpm_forward(np.ones((ny, nx), complex), dn, dx, dz, wavelength, n0, intensity=False)
    return out


def speckle_autocorrelation(intensity, max_lag):
    """C(d) for d = 0 .. max_lag, the mean of the x-lag and y-lag normalised
    circular autocovariances (sums written out, no FFT)."""
    I = np.asarray(intensity, float)
    d = I - I.mean()
    r0 = np.sum(d * d)
    return np.array([0.5 * (np.sum(d * np.roll(d, -s, axis=1)) + np.sum(d * np.roll(d, -s, axis=0)))
                     / r0 for s in range(max_lag + 1)])


def mean_free_paths(exit_plane_wave):
    """-ln |<u_N>|^2 for a unit plane wave at the entrance."""
    return float(-np.log(abs(np.mean(exit_plane_wave)) ** 2))
