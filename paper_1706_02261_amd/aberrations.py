"""Sample-induced aberrations as spatially resolved Zernike maps (main-text
paragraph on the light-sheet simulation).

Point sources on a grid at one depth of a dn volume ride in one multiplexed
field (as for the PSFs), are marched to the exit plane and brought back to
the source plane through the detection pupil; each source's window gives its
pupil field (``pupil_fields``) and the Zernike fit of the pupil phase gives
its aberration (``zernike_fit``), so a grid of sources gives a map of every
coefficient over the field of view (``zernike_map``).

Orchestration only: the march, the refocusing, the window DFTs and the fits
run in libbpm.so.
"""
from __future__ import annotations

import torch

from . import bpm as _bpm
from ._lib import check, lib
from .bpm import _need, _ptr, _stream_ptr
from .psfs import Optics


def pupil_fields(exit_field: torch.Tensor, sources: torch.Tensor, back_steps: int,
                 optics: Optics = Optics(), crop: int = 32, stream=None) -> torch.Tensor:
    """complex64 [n_src][crop][crop] pupil fields of the sources (int32
    [n_src][2] (y, x)) of a multiplexed run whose march started ``back_steps``
    slices before the exit plane."""
    _need(exit_field, "exit_field", torch.complex64)
    ny, nx = exit_field.shape
    _need(sources, "sources", torch.int32)
    n_src = sources.shape[0]
    out = torch.empty((n_src, crop, crop), dtype=torch.complex64, device=exit_field.device)
    ws = _bpm.workspace(int(lib().bpm_pupil_fields_workspace_size(nx, ny)) or 256,
                        exit_field.device)
    rc = lib().bpm_pupil_fields(_ptr(exit_field), nx, ny, float(optics.dx), float(optics.dz),
                                float(optics.wavelength), float(optics.n0), float(optics.na),
                                int(back_steps), _ptr(sources), n_src, int(crop), _ptr(out),
                                _ptr(ws), ws.numel(), _stream_ptr(stream))
    check(rc, "bpm_pupil_fields")
    return out


def zernike_fit(pupil: torch.Tensor, optics: Optics = Optics(), n_modes: int = 15,
                stream=None):
    """(coefficients float32 [n_src][n_modes] in radians, Noll order from
    piston; rms residual [n_src]) of pupil fields [n_src][crop][crop]."""
    _need(pupil, "pupil", torch.complex64)
    n_src, crop, _ = pupil.shape
    dev = pupil.device
    coeffs = torch.empty((n_src, n_modes), dtype=torch.float32, device=dev)
    rms = torch.empty((n_src,), dtype=torch.float32, device=dev)
    need = int(lib().bpm_zernike_workspace_size(crop, n_modes))
    ws = _bpm.workspace(need or 256, dev)
    rc = lib().bpm_zernike_fit(_ptr(pupil), n_src, crop, float(optics.dx),
                               float(optics.wavelength), float(optics.na), int(n_modes),
                               _ptr(coeffs), _ptr(rms), _ptr(ws), ws.numel(), _stream_ptr(stream))
    check(rc, "bpm_zernike_fit")
    return coeffs, rms


def zernike_map(dn: torch.Tensor, depth: int, pitch: int = 32, optics: Optics = Optics(),
                n_modes: int = 15, crop: int = 32, offset=None):
    """Aberration maps of sources on a ``pitch`` grid at slice ``depth`` of
    ``dn`` [nz][ny][nx] (one multiplexed march).  Returns (coefficient maps
    float32 [n_modes][gy][gx], rms map [gy][gx], sources int32 [gy*gx][2])."""
    _need(dn, "dn", torch.float32)
    nz, ny, nx = dn.shape
    if not 0 <= depth < nz:
        raise ValueError(f"depth={depth} must be in [0, {nz})")
    if pitch < crop:
        raise ValueError(f"pitch={pitch} must be at least the window crop={crop}")
    oy, ox = (pitch // 2, pitch // 2) if offset is None else offset
    dev = dn.device
    ys = torch.arange(oy % pitch, ny, pitch, dtype=torch.int32, device=dev)
    xs = torch.arange(ox % pitch, nx, pitch, dtype=torch.int32, device=dev)
    src = torch.stack(torch.meshgrid(ys, xs, indexing="ij"), -1).reshape(-1, 2).contiguous()
    u0 = _bpm.point_sources(src, nx, ny, optics.dx, optics.wavelength, optics.n0, optics.na, 0.0)
    exit_field, _ = _bpm.propagate(u0, dn[depth:], optics.dx, optics.dz, optics.wavelength,
                                   optics.n0, intensity=False)
    X = pupil_fields(exit_field, src, nz - depth, optics, crop)
    c, rms = zernike_fit(X, optics, n_modes)
    gy, gx = ys.numel(), xs.numel()
    return c.T.reshape(n_modes, gy, gx), rms.reshape(gy, gx), src
