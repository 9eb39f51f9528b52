"""Adaptive optics through scattering tissue (main-text paragraph on adaptive
optics; Fig. 2c, d).

* ``guide_star_phase`` -- conjugating the wavefront of a point-like guide star
  at the focus: one linear adjoint march (M^H e_f, no forward march) and the
  phase kernel give the entrance pupil phase phi* that maximises the focus
  intensity for a fixed pupil amplitude.
* ``optimize_pupil`` -- the same problem, and sums over several foci, by
  gradient ascent: forward march, linear adjoint of the focus amplitudes,
  pupil-phase gradient and an Adam step per iteration.
* ``memory_effect`` -- the corrected entrance field shifted laterally (the
  phase kernel's tilt), marched in lockstep batches; the persistence
  P(s) = I_s(x_f + s) / I_0(x_f) against ``speckle_autocorrelation`` of the
  exit intensity of a plane wave, and ``mean_free_paths`` of the tissue.

Marches, adjoints, FFTs, phases and optimiser steps run in libbpm.so; what
torch does here is allocation, a one-pixel source, |u|^2 and means of the
results.
"""
from __future__ import annotations

import dataclasses

import torch

from . import bpm as _bpm
from .bpm import _need


@dataclasses.dataclass(frozen=True)
class Optics:
    """Sampling and optics of an adaptive-optics problem (micrometres)."""
    dx: float = 0.2
    dz: float = 0.2
    wavelength: float = 0.5
    n0: float = 1.36


def _point(ny, nx, focus, device, value=1.0):
    e = torch.zeros((ny, nx), dtype=torch.complex64, device=device)
    e[focus[0], focus[1]] = value
    return e


def guide_star_gradient(dn: torch.Tensor, focus, optics: Optics = Optics(), ws=None):
    """G = DFT2(M^H e_f) / (nx ny): the entrance-spectrum gradient of the focus
    amplitude, from one adjoint march of a point at ``focus`` = (y, x) of the
    exit plane of ``dn`` [steps][ny][nx]."""
    _need(dn, "dn", torch.float32)
    _, ny, nx = dn.shape
    e = _point(ny, nx, focus, dn.device)
    _, gs, _ = _bpm.adjoint(None, dn, optics.dx, optics.dz, optics.wavelength, optics.n0,
                            grad_field_out=e, want_field=False, want_spectrum=True,
                            want_dn=False, ws=ws)
    return gs


def guide_star_gradients(dn: torch.Tensor, foci, optics: Optics = Optics()):
    """``guide_star_gradient`` of several foci through the same ``dn``, the
    adjoints of up to eight guide stars in each lockstep launch (bitwise the
    separate results).  Returns one G per focus."""
    _need(dn, "dn", torch.float32)
    _, ny, nx = dn.shape
    out = []
    for i in range(0, len(foci), 8):
        jobs = [dict(dn=dn, grad_field_out=_point(ny, nx, f, dn.device), want_field=False,
                     want_spectrum=True, want_dn=False) for f in foci[i:i + 8]]
        out += [gs for _, gs, _ in _bpm.adjoint_batch(jobs, optics.dx, optics.dz,
                                                      optics.wavelength, optics.n0)]
    return out


def guide_star_phase(dn: torch.Tensor, focus, z_focus: float, optics: Optics = Optics(),
                     shift=(0.0, 0.0)):
    """Corrected pupil phase phi* = arg G + kz z_focus (minus the tilt of a
    ``shift`` = (x, y) micrometres of the entrance field) and G itself."""
    gs = guide_star_gradient(dn, focus, optics)
    return _bpm.guide_star_phase(gs, optics.dx, optics.wavelength, optics.n0, z_focus,
                                 shift=shift), gs


def aim_phase(ny: int, nx: int, focus, optics: Optics = Optics(), device="cuda"):
    """-(kx x_f + ky y_f): the wavefront that focuses on ``focus`` in a clear
    medium (the guide-star phase of G = 1 with z_focus = 0, shifted to x_f)."""
    ones = torch.ones((ny, nx), dtype=torch.complex64, device=device)
    return _bpm.guide_star_phase(ones, optics.dx, optics.wavelength, optics.n0, 0.0,
                                 shift=(focus[1] * optics.dx, focus[0] * optics.dx))


def exit_field(amplitude: torch.Tensor, phase: torch.Tensor, dn: torch.Tensor, z_focus: float,
               optics: Optics = Optics(), ws=None):
    """Exit-plane field of the entrance spectrum A exp(i phi) exp(-i kz z_focus)."""
    spec = _bpm.pupil_spectrum(amplitude, phase, optics.dx, optics.wavelength, optics.n0, z_focus)
    u0 = _bpm.fft2(spec, inverse=True)
    out, _ = _bpm.propagate(u0, dn, optics.dx, optics.dz, optics.wavelength, optics.n0,
                            intensity=False, ws=ws)
    return out


def optimum_intensity(amplitude: torch.Tensor, gs: torch.Tensor) -> float:
    """(sum A |G|)^2, the focus intensity of the guide-star correction."""
    return float((amplitude.double() * gs.abs().double()).sum()) ** 2


class FocusProblem:
    """The multi-focus objective L = -sum_f |u(x_f)|^2 on one tissue, with its
    buffers (workspace, adjoint source) kept across calls of ``gradient``."""

    def __init__(self, dn, foci):
        _, ny, nx = dn.shape
        dev = dn.device
        self.fy = torch.tensor([f[0] for f in foci], dtype=torch.long, device=dev)
        self.fx = torch.tensor([f[1] for f in foci], dtype=torch.long, device=dev)
        self.ws = _bpm.workspace(max(_bpm.workspace_size(nx, ny, dn.shape[0]),
                                     _bpm.adjoint_workspace_size(nx, ny, dn.shape[0])), dev)
        self.g_out = torch.zeros((ny, nx), dtype=torch.complex64, device=dev)

    def gradient(self, amplitude, phase, dn, z_focus, optics):
        """Focus intensities and dL/dphi: forward march, dL/du_N =
        -2 sum_f u(x_f) e_f, one linear adjoint march, Im(dL/dU0 conj(U0))."""
        spec = _bpm.pupil_spectrum(amplitude, phase, optics.dx, optics.wavelength, optics.n0,
                                   z_focus)
        u0 = _bpm.fft2(spec, inverse=True)
        out, _ = _bpm.propagate(u0, dn, optics.dx, optics.dz, optics.wavelength, optics.n0,
                                intensity=False, ws=self.ws)
        uf = out[self.fy, self.fx]
        self.g_out.zero_()
        self.g_out[self.fy, self.fx] = -2.0 * uf
        _, gs, _ = _bpm.adjoint(None, dn, optics.dx, optics.dz, optics.wavelength, optics.n0,
                                grad_field_out=self.g_out, want_field=False, want_spectrum=True,
                                want_dn=False, ws=self.ws)
        return uf.abs() ** 2, _bpm.pupil_phase_grad(gs, spec)


def focus_gradient(amplitude: torch.Tensor, phase: torch.Tensor, dn: torch.Tensor, foci,
                   z_focus: float, optics: Optics = Optics()):
    """(focus intensities [n_foci], dL/dphi [ny][nx]) of L = -sum_f |u(x_f)|^2
    for ``foci`` a list of (y, x) exit-plane pixels."""
    _need(amplitude, "amplitude", torch.float32)
    _need(phase, "phase", torch.float32)
    _need(dn, "dn", torch.float32)
    return FocusProblem(dn, foci).gradient(amplitude, phase, dn, z_focus, optics)


def optimize_pupil(amplitude: torch.Tensor, dn: torch.Tensor, foci, z_focus: float,
                   optics: Optics = Optics(), iters: int = 100, lr: float = 0.1,
                   phase0: torch.Tensor | None = None):
    """Maximise sum_f |u(x_f)|^2 over the pupil phase by Adam on
    ``focus_gradient``.  Returns (phase, history [iters][n_foci] of the focus
    intensities before each update)."""
    _need(amplitude, "amplitude", torch.float32)
    _need(dn, "dn", torch.float32)
    _, ny, nx = dn.shape
    dev = dn.device
    phase = (torch.zeros((ny, nx), dtype=torch.float32, device=dev) if phase0 is None
             else phase0.clone().contiguous())
    m = torch.zeros_like(phase)
    v = torch.zeros_like(phase)
    prob = FocusProblem(dn, foci)
    hist = torch.empty((iters, len(foci)), dtype=torch.float32, device=dev)
    for t in range(1, iters + 1):
        hist[t - 1], gphi = prob.gradient(amplitude, phase, dn, z_focus, optics)
        _bpm.adam_step(phase, gphi, m, v, lr, t)
    return phase, hist


def memory_effect(amplitude: torch.Tensor, gs: torch.Tensor, dn: torch.Tensor, focus, shifts,
                  z_focus: float, optics: Optics = Optics()):
    """Persistence of the shifted correction: for each integer pixel shift
    s = (sy, sx), the corrected phase tilted to move the entrance field by s,
    marched (lockstep batches of up to eight), read at x_f + s, over the
    unshifted focus intensity.  Returns (P [len(shifts)] float64 on the host,
    unshifted focus intensity)."""
    _need(dn, "dn", torch.float32)
    _, ny, nx = dn.shape
    cases = [(0, 0)] + [tuple(int(c) for c in s) for s in shifts]
    fields = []
    for sy, sx in cases:
        ph = _bpm.guide_star_phase(gs, optics.dx, optics.wavelength, optics.n0, z_focus,
                                   shift=(sx * optics.dx, sy * optics.dx))
        spec = _bpm.pupil_spectrum(amplitude, ph, optics.dx, optics.wavelength, optics.n0,
                                   z_focus)
        fields.append(_bpm.fft2(spec, inverse=True))
    vals = []
    for b in range(0, len(fields), 8):
        jobs = [dict(field=f, dn=dn, dx=optics.dx, dz=optics.dz, wavelength=optics.wavelength,
                     n0=optics.n0, out=f, intensity=False) for f in fields[b:b + 8]]
        for (out, _), (sy, sx) in zip(_bpm.propagate_batch(jobs), cases[b:b + 8]):
            vals.append(out[(focus[0] + sy) % ny, (focus[1] + sx) % nx].abs() ** 2)
    vals = torch.stack(vals).double().cpu()
    return (vals[1:] / vals[0]).numpy(), float(vals[0])


def plane_wave_exit(dn: torch.Tensor, optics: Optics = Optics()):
    """Exit field of a unit plane wave at normal incidence."""
    _need(dn, "dn", torch.float32)
    _, ny, nx = dn.shape
    u0 = torch.ones((ny, nx), dtype=torch.complex64, device=dn.device)
    out, _ = _bpm.propagate(u0, dn, optics.dx, optics.dz, optics.wavelength, optics.n0,
                            intensity=False)
    return out


def speckle_autocorrelation(intensity: torch.Tensor, max_lag: int):
    """C(d), d = 0 .. max_lag: the normalised circular autocovariance of an
    intensity pattern, mean of the x and y lags, by the Wiener-Khinchin
    theorem (two library FFTs).  Returns float64 on the host."""
    _need(intensity, "intensity", torch.float32)
    d = (intensity - intensity.mean()).to(torch.complex64).contiguous()
    F = _bpm.fft2(d)
    R = _bpm.fft2((F.abs() ** 2).to(torch.complex64).contiguous(), inverse=True).real.double()
    R = (R / R[0, 0]).cpu()
    return (0.5 * (R[0, :max_lag + 1] + R[:max_lag + 1, 0])).numpy()


def mean_free_paths(exit_plane_wave: torch.Tensor) -> float:
    """-ln |<u_N>|^2 of a unit plane wave: the depth in scattering mean free
    paths (the ballistic power decays as exp(-z / l_s)); inf when no
    ballistic light is left."""
    import math
    p = float(exit_plane_wave.mean().abs()) ** 2
    return math.inf if p == 0.0 else -math.log(p)
