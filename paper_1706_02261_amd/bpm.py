"""Torch-facing binding of the march entry points (argument marshalling only)."""
from __future__ import annotations

import torch

from . import _lib
from ._lib import check, lib


def _stream_ptr(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _need(t: torch.Tensor, name: str, dtype, shape=None) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU device, got {t.device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _ptr(t):
    return None if t is None else t.data_ptr()


def workspace_size(nx: int, ny: int, steps: int, adjoint: bool = False) -> int:
    n = lib().bpm_workspace_size(nx, ny, steps,
                                 _lib.BPM_WS_ADJOINT if adjoint else _lib.BPM_WS_FORWARD)
    if n == 0:
        raise _lib.BpmError(_lib.BPM_ERR_UNSUPPORTED_SIZE,
                            f"no workspace size for nx={nx} ny={ny} steps={steps}")
    return int(n)


def workspace(nbytes: int, device) -> torch.Tensor:
    """Caller-owned device workspace (torch's allocator aligns to 512 bytes)."""
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def propagate(field: torch.Tensor, dn: torch.Tensor, dx: float, dz: float,
              wavelength: float, n0: float, intensity: bool = True,
              out: torch.Tensor | None = None, intensity_out: torch.Tensor | None = None,
              ws: torch.Tensor | None = None, stream=None):
    """March ``field`` (complex64 [ny][nx]) through ``dn`` (float32 [steps][ny][nx]).

    Returns ``(field_out, intensity)``; ``intensity`` is the float32
    [steps][ny][nx] volume |u_{j+1}|^2 or None when ``intensity`` is False.
    """
    _need(field, "field", torch.complex64)
    ny, nx = field.shape
    _need(dn, "dn", torch.float32)
    if dn.dim() != 3 or tuple(dn.shape[1:]) != (ny, nx):
        raise ValueError(f"dn has shape {tuple(dn.shape)}, expected [steps][{ny}][{nx}]")
    steps = dn.shape[0]
    if out is None:
        out = torch.empty_like(field)
    _need(out, "out", torch.complex64, (ny, nx))
    if intensity and intensity_out is None:
        intensity_out = torch.empty((steps, ny, nx), dtype=torch.float32, device=field.device)
    if not intensity:
        intensity_out = None
    if intensity_out is not None:
        _need(intensity_out, "intensity_out", torch.float32, (steps, ny, nx))
    need = workspace_size(nx, ny, steps)
    if ws is None:
        ws = workspace(need, field.device)
    rc = lib().bpm_propagate(_ptr(field), _ptr(dn), nx, ny, steps, float(dx), float(dz),
                             float(wavelength), float(n0), _ptr(out), _ptr(intensity_out),
                             _ptr(ws), ws.numel(), _stream_ptr(stream))
    check(rc, "bpm_propagate")
    return out, intensity_out
