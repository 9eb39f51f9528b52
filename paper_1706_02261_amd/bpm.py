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


def slice_means(dn: torch.Tensor, stream=None) -> torch.Tensor:
    """Mean of every slice of ``dn`` ([steps][ny][nx] float32) -> [steps]."""
    _need(dn, "dn", torch.float32)
    if dn.dim() != 3:
        raise ValueError("dn must be [steps][ny][nx]")
    steps, ny, nx = dn.shape
    out = torch.empty(steps, dtype=torch.float32, device=dn.device)
    check(lib().bpm_slice_means(_ptr(dn), nx, ny, steps, _ptr(out), _stream_ptr(stream)),
          "bpm_slice_means")
    return out


def propagate_adapted(field: torch.Tensor, dn: torch.Tensor, dx: float, dz: float,
                      wavelength: float, n0: float, dn_ref: torch.Tensor | None = None,
                      intensity: bool = True, out: torch.Tensor | None = None,
                      ws: torch.Tensor | None = None, stream=None):
    """March with the locally adapted expansion: slice j about n0 + dn_ref[j]
    (default: the slice means of ``dn``).  Returns (field_out, intensity or
    None, dn_ref)."""
    _need(field, "field", torch.complex64)
    ny, nx = field.shape
    _need(dn, "dn", torch.float32)
    if dn.dim() != 3 or tuple(dn.shape[1:]) != (ny, nx):
        raise ValueError(f"dn has shape {tuple(dn.shape)}, expected [steps][{ny}][{nx}]")
    steps = dn.shape[0]
    if dn_ref is None:
        dn_ref = slice_means(dn, stream=stream)
    _need(dn_ref, "dn_ref", torch.float32, (steps,))
    if out is None:
        out = torch.empty_like(field)
    _need(out, "out", torch.complex64, (ny, nx))
    inten = (torch.empty((steps, ny, nx), dtype=torch.float32, device=field.device)
             if intensity else None)
    if ws is None:
        ws = workspace(workspace_size(nx, ny, steps), field.device)
    rc = lib().bpm_propagate_adapted(_ptr(field), _ptr(dn), _ptr(dn_ref), nx, ny, steps,
                                     float(dx), float(dz), float(wavelength), float(n0), _ptr(out),
                                     _ptr(inten), _ptr(ws), ws.numel(), _stream_ptr(stream))
    check(rc, "bpm_propagate_adapted")
    return out, inten, dn_ref


def propagate_noalloc(field: torch.Tensor, dn: torch.Tensor, dx: float, dz: float,
                      wavelength: float, n0: float, out: torch.Tensor,
                      intensity_out: torch.Tensor | None = None, stream=None):
    """bpm_propagate_noalloc: ``propagate`` into caller-given ``out`` (and
    ``intensity_out`` or None) with the library's own per-GPU plan memory; no
    allocation of any kind (fields up to 1024 x 1024)."""
    _need(field, "field", torch.complex64)
    ny, nx = field.shape
    _need(dn, "dn", torch.float32)
    if dn.dim() != 3 or tuple(dn.shape[1:]) != (ny, nx):
        raise ValueError(f"dn has shape {tuple(dn.shape)}, expected [steps][{ny}][{nx}]")
    steps = dn.shape[0]
    _need(out, "out", torch.complex64, (ny, nx))
    if intensity_out is not None:
        _need(intensity_out, "intensity_out", torch.float32, (steps, ny, nx))
    rc = lib().bpm_propagate_noalloc(_ptr(field), _ptr(dn), nx, ny, steps, float(dx), float(dz),
                                     float(wavelength), float(n0), _ptr(out),
                                     _ptr(intensity_out), _stream_ptr(stream))
    check(rc, "bpm_propagate_noalloc")
    return out, intensity_out


def workspace_status(ws: torch.Tensor, stream=None) -> None:
    """Raise BpmError (BPM_ERR_DEVICE) if a wait of a kernel that used ``ws``
    gave up since the last query (its outputs are not valid); synchronises the
    stream and resets the record."""
    _need(ws, "ws", torch.uint8)
    check(lib().bpm_workspace_status(_ptr(ws), ws.numel(), _stream_ptr(stream)),
          "bpm_workspace_status")


def set_wait_limit(polls: int = 0) -> None:
    """Bound on the polls of one grid-barrier or queue wait (0: the default)."""
    check(lib().bpm_set_wait_limit(int(polls)), "bpm_set_wait_limit")


def adjoint_workspace_size(nx: int, ny: int, steps: int, checkpoint_every: int = 0) -> int:
    n = lib().bpm_adjoint_workspace_size(nx, ny, steps, checkpoint_every)
    if n == 0:
        raise _lib.BpmError(_lib.BPM_ERR_INVALID_ARG,
                            f"no adjoint workspace for nx={nx} ny={ny} steps={steps} "
                            f"checkpoint_every={checkpoint_every}")
    return int(n)


def adjoint(field: torch.Tensor, dn: torch.Tensor, dx: float, dz: float, wavelength: float,
            n0: float, grad_field_out: torch.Tensor | None = None,
            grad_intensity: torch.Tensor | None = None, want_field: bool = True,
            want_spectrum: bool = False, want_dn: bool = True, checkpoint_every: int = 0,
            ws: torch.Tensor | None = None, stream=None):
    """Gradients through ``propagate`` (PyTorch's complex convention).

    Returns ``(grad_field_in, grad_spectrum_in, grad_dn)`` with None for the
    ones not requested.  ``field`` may be None when neither intensity nor dn
    gradients are wanted (``grad_intensity`` None, ``want_dn`` False): the
    result is then M^H grad_field_out and the forward march is skipped."""
    _need(dn, "dn", torch.float32)
    if field is None:
        if grad_field_out is None or grad_intensity is not None or want_dn:
            raise ValueError("field may be None only for the linear adjoint "
                             "(grad_field_out given, no grad_intensity, want_dn False)")
        ny, nx = grad_field_out.shape
    else:
        _need(field, "field", torch.complex64)
        ny, nx = field.shape
    if dn.dim() != 3 or tuple(dn.shape[1:]) != (ny, nx):
        raise ValueError(f"dn has shape {tuple(dn.shape)}, expected [steps][{ny}][{nx}]")
    steps = dn.shape[0]
    if grad_field_out is not None:
        _need(grad_field_out, "grad_field_out", torch.complex64, (ny, nx))
    if grad_intensity is not None:
        _need(grad_intensity, "grad_intensity", torch.float32, (steps, ny, nx))
    dev = dn.device
    g0 = torch.empty((ny, nx), dtype=torch.complex64, device=dev) if want_field else None
    gs = torch.empty((ny, nx), dtype=torch.complex64, device=dev) if want_spectrum else None
    gdn = torch.empty((steps, ny, nx), dtype=torch.float32, device=dev) if want_dn else None
    need = adjoint_workspace_size(nx, ny, steps, checkpoint_every)
    if ws is None:
        ws = workspace(need, dev)
    rc = lib().bpm_adjoint(_ptr(field), _ptr(dn), nx, ny, steps, float(dx), float(dz),
                           float(wavelength), float(n0), _ptr(grad_field_out),
                           _ptr(grad_intensity), _ptr(g0), _ptr(gs), _ptr(gdn),
                           int(checkpoint_every), _ptr(ws), ws.numel(), _stream_ptr(stream))
    check(rc, "bpm_adjoint")
    return g0, gs, gdn


def adjoint_batch_workspace_size(n_fields: int, nx: int, ny: int, steps: int,
                                 checkpoint_every: int = 0) -> int:
    n = lib().bpm_adjoint_batch_workspace_size(n_fields, nx, ny, steps, checkpoint_every)
    if n == 0:
        raise _lib.BpmError(_lib.BPM_ERR_INVALID_ARG,
                            f"no adjoint workspace for {n_fields} fields nx={nx} ny={ny} "
                            f"steps={steps} checkpoint_every={checkpoint_every}")
    return int(n)


def adjoint_batch(jobs, dx: float, dz: float, wavelength: float, n0: float,
                  checkpoint_every: int = 0, ws: torch.Tensor | None = None, stream=None):
    """Several adjoints of one geometry in one lockstep launch (the fields
    share each grid barrier); bitwise the results of separate ``adjoint``
    calls.  Each job is a dict with ``dn`` and the optional ``field``,
    ``grad_field_out``, ``grad_intensity``, ``want_field`` (default True),
    ``want_spectrum`` (False) and ``want_dn`` (True) of ``adjoint``; at most
    8 jobs.  Returns one ``(grad_field_in, grad_spectrum_in, grad_dn)`` per
    job."""
    if not 1 <= len(jobs) <= _lib.BPM_MAX_LOCKSTEP_FIELDS:
        raise ValueError(f"{len(jobs)} jobs: 1 to {_lib.BPM_MAX_LOCKSTEP_FIELDS} per launch")
    shape = None
    table = (_lib.AdjointJob * len(jobs))()
    outs = []
    for k, j in enumerate(jobs):
        dn = j["dn"]
        _need(dn, "dn", torch.float32)
        if dn.dim() != 3:
            raise ValueError(f"job {k}: dn must be [steps][ny][nx]")
        if shape is None:
            shape = tuple(dn.shape)
        elif tuple(dn.shape) != shape:
            raise ValueError(f"job {k}: dn has shape {tuple(dn.shape)}, job 0 {shape}")
        steps, ny, nx = shape
        field, gout, gI = j.get("field"), j.get("grad_field_out"), j.get("grad_intensity")
        want_dn = j.get("want_dn", True)
        if field is None and (gout is None or gI is not None or want_dn):
            raise ValueError(f"job {k}: field may be None only for the linear adjoint")
        if field is not None:
            _need(field, "field", torch.complex64, (ny, nx))
        if gout is not None:
            _need(gout, "grad_field_out", torch.complex64, (ny, nx))
        if gI is not None:
            _need(gI, "grad_intensity", torch.float32, (steps, ny, nx))
        dev = dn.device
        g0 = (torch.empty((ny, nx), dtype=torch.complex64, device=dev)
              if j.get("want_field", True) else None)
        gs = (torch.empty((ny, nx), dtype=torch.complex64, device=dev)
              if j.get("want_spectrum", False) else None)
        gdn = torch.empty((steps, ny, nx), dtype=torch.float32, device=dev) if want_dn else None
        table[k] = _lib.AdjointJob(_ptr(field), _ptr(dn), _ptr(gout), _ptr(gI), _ptr(g0),
                                   _ptr(gs), _ptr(gdn))
        outs.append((g0, gs, gdn))
    steps, ny, nx = shape
    need = adjoint_batch_workspace_size(len(jobs), nx, ny, steps, checkpoint_every)
    if ws is None:
        ws = workspace(need, jobs[0]["dn"].device)
    rc = lib().bpm_adjoint_batch(table, len(jobs), nx, ny, steps, float(dx), float(dz),
                                 float(wavelength), float(n0), int(checkpoint_every), _ptr(ws),
                                 ws.numel(), _stream_ptr(stream))
    check(rc, "bpm_adjoint_batch")
    return outs


def fft2(x: torch.Tensor, inverse: bool = False, out: torch.Tensor | None = None, stream=None):
    """Natural-order 2-D DFT (numpy's fft2 / ifft2 conventions) of a complex64 [ny][nx]."""
    _need(x, "x", torch.complex64)
    ny, nx = x.shape
    if out is None:
        out = torch.empty_like(x)
    _need(out, "out", torch.complex64, (ny, nx))
    ws = workspace(lib().bpm_fft2_workspace_size(nx, ny), x.device)
    rc = lib().bpm_fft2(_ptr(x), _ptr(out), nx, ny, 1 if inverse else 0, _ptr(ws), ws.numel(),
                        _stream_ptr(stream))
    check(rc, "bpm_fft2")
    return out


def pupil_spectrum(amplitude: torch.Tensor, phase: torch.Tensor, dx: float, wavelength: float,
                   n0: float, z_focus: float, stream=None) -> torch.Tensor:
    """U0 = A exp(i phi) exp(-i kz z_focus) on the natural DFT grid."""
    _need(amplitude, "amplitude", torch.float32)
    ny, nx = amplitude.shape
    _need(phase, "phase", torch.float32, (ny, nx))
    out = torch.empty((ny, nx), dtype=torch.complex64, device=amplitude.device)
    rc = lib().bpm_pupil_spectrum(_ptr(amplitude), _ptr(phase), nx, ny, float(dx),
                                  float(wavelength), float(n0), float(z_focus), _ptr(out),
                                  _stream_ptr(stream))
    check(rc, "bpm_pupil_spectrum")
    return out


def guide_star_phase(grad_spectrum: torch.Tensor, dx: float, wavelength: float, n0: float,
                     z_focus: float, shift=(0.0, 0.0), out: torch.Tensor | None = None,
                     stream=None) -> torch.Tensor:
    """Pupil phase arg(G) + kz z_focus - kx shift_x - ky shift_y in [-pi, pi)
    from the spectrum gradient G of a point at the focus (``shift`` = (x, y)
    in micrometres moves the corrected entrance field)."""
    _need(grad_spectrum, "grad_spectrum", torch.complex64)
    ny, nx = grad_spectrum.shape
    if out is None:
        out = torch.empty((ny, nx), dtype=torch.float32, device=grad_spectrum.device)
    _need(out, "out", torch.float32, (ny, nx))
    rc = lib().bpm_guide_star_phase(_ptr(grad_spectrum), nx, ny, float(dx), float(wavelength),
                                    float(n0), float(z_focus), float(shift[0]), float(shift[1]),
                                    _ptr(out), _stream_ptr(stream))
    check(rc, "bpm_guide_star_phase")
    return out


def adam_step(params: torch.Tensor, grads: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
              lr: float, step: int, stream=None) -> None:
    """One Adam update of float32 ``params`` in place (moments m, v in place;
    1-based ``step``)."""
    _need(params, "params", torch.float32)
    for t, name in ((grads, "grads"), (m, "m"), (v, "v")):
        _need(t, name, torch.float32, tuple(params.shape))
    rc = lib().bpm_adam_step(_ptr(params), _ptr(grads), _ptr(m), _ptr(v), params.numel(),
                             float(lr), int(step), _stream_ptr(stream))
    check(rc, "bpm_adam_step")


def pupil_phase_grad(grad_spectrum: torch.Tensor, spectrum: torch.Tensor, stream=None):
    """dL/dphi = Im(dL/dU0 conj(U0))."""
    _need(spectrum, "spectrum", torch.complex64)
    ny, nx = spectrum.shape
    _need(grad_spectrum, "grad_spectrum", torch.complex64, (ny, nx))
    out = torch.empty((ny, nx), dtype=torch.float32, device=spectrum.device)
    rc = lib().bpm_pupil_phase_grad(_ptr(grad_spectrum), _ptr(spectrum), nx, ny, _ptr(out),
                                    _stream_ptr(stream))
    check(rc, "bpm_pupil_phase_grad")
    return out


class BPMFunction(torch.autograd.Function):
    """(field, dn) -> (field_out, intensity) with the hand-written adjoint march
    (checkpointed recomputation) as backward."""

    @staticmethod
    def forward(ctx, field, dn, dx, dz, wavelength, n0, checkpoint_every=0):
        field = field.contiguous()
        dn = dn.contiguous()
        out, inten = propagate(field, dn, dx, dz, wavelength, n0, intensity=True)
        ctx.save_for_backward(field, dn)
        ctx.geom = (dx, dz, wavelength, n0, checkpoint_every)
        return out, inten

    @staticmethod
    def backward(ctx, g_out, g_inten):
        field, dn = ctx.saved_tensors
        dx, dz, wavelength, n0, ck = ctx.geom
        g_out = None if g_out is None else g_out.contiguous()
        g_inten = None if g_inten is None else g_inten.contiguous()
        g0, _, gdn = adjoint(field, dn, dx, dz, wavelength, n0, grad_field_out=g_out,
                             grad_intensity=g_inten, want_field=ctx.needs_input_grad[0],
                             want_dn=ctx.needs_input_grad[1], checkpoint_every=ck)
        return g0, gdn, None, None, None, None, None


class PupilBPMFunction(torch.autograd.Function):
    """(pupil phase, dn) -> (field_out, intensity) for the entry field
    u0 = IDFT2(A exp(i phi) exp(-i kz z_focus)); backward gives dL/dphi (the
    adaptive-optics correction) and dL/ddn."""

    @staticmethod
    def forward(ctx, phase, amplitude, dn, dx, dz, wavelength, n0, z_focus, checkpoint_every=0):
        phase = phase.contiguous()
        amplitude = amplitude.contiguous()
        dn = dn.contiguous()
        spec = pupil_spectrum(amplitude, phase, dx, wavelength, n0, z_focus)
        u0 = fft2(spec, inverse=True)
        out, inten = propagate(u0, dn, dx, dz, wavelength, n0, intensity=True)
        ctx.save_for_backward(spec, u0, dn)
        ctx.geom = (dx, dz, wavelength, n0, checkpoint_every)
        return out, inten

    @staticmethod
    def backward(ctx, g_out, g_inten):
        spec, u0, dn = ctx.saved_tensors
        dx, dz, wavelength, n0, ck = ctx.geom
        g_out = None if g_out is None else g_out.contiguous()
        g_inten = None if g_inten is None else g_inten.contiguous()
        _, gspec, gdn = adjoint(u0, dn, dx, dz, wavelength, n0, grad_field_out=g_out,
                                grad_intensity=g_inten, want_field=False, want_spectrum=True,
                                want_dn=ctx.needs_input_grad[2], checkpoint_every=ck)
        gphi = pupil_phase_grad(gspec, spec) if ctx.needs_input_grad[0] else None
        return gphi, None, gdn, None, None, None, None, None, None


def _batch_table(jobs):
    """ctypes job array and (out, intensity) tensors of a batch."""
    arr = (_lib.Job * len(jobs))()
    results = []
    dev = None
    for i, j in enumerate(jobs):
        f, d = j["field"], j["dn"]
        _need(f, f"jobs[{i}].field", torch.complex64)
        _need(d, f"jobs[{i}].dn", torch.float32)
        ny, nx = f.shape
        if d.dim() != 3 or tuple(d.shape[1:]) != (ny, nx):
            raise ValueError(f"jobs[{i}].dn has shape {tuple(d.shape)}, expected [steps][{ny}][{nx}]")
        steps = d.shape[0]
        out = j.get("out")
        if out is None:
            out = torch.empty_like(f)
        _need(out, f"jobs[{i}].out", torch.complex64, (ny, nx))
        inten = j.get("intensity_out")
        if inten is None and j.get("intensity", True):
            inten = torch.empty((steps, ny, nx), dtype=torch.float32, device=f.device)
        if inten is not None:
            _need(inten, f"jobs[{i}].intensity_out", torch.float32, (steps, ny, nx))
        arr[i] = _lib.Job(f.data_ptr(), d.data_ptr(), nx, ny, steps, float(j["dx"]),
                          float(j["dz"]), float(j["wavelength"]), float(j["n0"]),
                          out.data_ptr(), 0 if inten is None else inten.data_ptr(),
                          int(j.get("clear_steps", 0)))
        results.append((out, inten))
        dev = f.device
    need = lib().bpm_batch_workspace_size(arr, len(jobs))
    if need == 0:
        raise _lib.BpmError(_lib.BPM_ERR_UNSUPPORTED_SIZE, "unsupported job in batch")
    return arr, results, int(need), dev


def propagate_batch(jobs, ws: torch.Tensor | None = None, stream=None):
    """Run an uneven batch of marches in one persistent launch.

    ``jobs``: sequence of dicts with keys field, dn, dx, dz, wavelength, n0 and
    optional out, intensity (bool, default True), intensity_out and
    clear_steps (leading steps in the background medium, whose dn slices are
    not read; default 0).  Returns a list of (field_out, intensity) per job."""
    if len(jobs) == 0:
        return []
    arr, results, need, dev = _batch_table(jobs)
    if ws is None:
        ws = workspace(need, dev)
    rc = lib().bpm_propagate_batch(arr, len(jobs), _ptr(ws), ws.numel(), _stream_ptr(stream))
    check(rc, "bpm_propagate_batch")
    return results


PHASES = ("setup", "head", "column", "row", "drain", "wait")


def march_phase_times(jobs, ws: torch.Tensor | None = None, stream=None):
    """The lockstep march of ``propagate_batch`` (1-8 jobs of one geometry)
    with per-workgroup phase timers.  Returns (results, times) where times is a
    dict: "workgroups", "steps", "fields" and, per phase name in PHASES, a
    float64 tensor [workgroups] of seconds."""
    arr, results, need, dev = _batch_table(jobs)
    if ws is None:
        ws = workspace(need, dev)
    t = torch.empty(_lib.PHASE_TIMER_WORDS, dtype=torch.int64, device=dev)
    rc = lib().bpm_march_phase_times(arr, len(jobs), _ptr(ws), ws.numel(), _ptr(t),
                                     t.numel() * 8, _stream_ptr(stream))
    check(rc, "bpm_march_phase_times")
    h = t.cpu()
    G, rate, steps, fields = (int(h[k]) for k in range(4))
    rec = h[8:8 + 8 * G].view(G, 8).double() / rate
    times = {"workgroups": G, "steps": steps, "fields": fields}
    for k, name in enumerate(PHASES):
        times[name] = rec[:, k]
    return results, times


class PreparedBatch:
    """An uneven batch whose tables sit in its own workspace, so that
    ``launch()`` issues device work only and can be captured into a graph
    (``torch.cuda.graph``) and replayed.  Inputs and outputs are the tensors
    given (or allocated) here; a replay reads the inputs' current contents."""

    def __init__(self, jobs, stream=None):
        if len(jobs) == 0:
            raise ValueError("a prepared batch needs at least one job")
        self._jobs = list(jobs)  # keeps the input tensors alive
        self._arr, self.results, need, dev = _batch_table(self._jobs)
        self.ws = workspace(need, dev)
        check(lib().bpm_batch_upload(self._arr, len(self._jobs), _ptr(self.ws), self.ws.numel(),
                                     _stream_ptr(stream)), "bpm_batch_upload")

    def launch(self, stream=None):
        check(lib().bpm_batch_launch(self._arr, len(self._jobs), _ptr(self.ws), self.ws.numel(),
                                     _stream_ptr(stream)), "bpm_batch_launch")
        return self.results


def psf_readout(exit_field: torch.Tensor, sources: torch.Tensor, dx: float, dz: float,
                wavelength: float, n0: float, na: float, back_steps: int, planes: int = 32,
                crop: int = 32, scale: float = 1.0, ws: torch.Tensor | None = None, stream=None):
    """Refocused PSF stacks [n_src][planes][crop][crop] of a multiplexed run.

    ``sources``: int32 [n_src][2] (y, x) pixel positions on the device."""
    _need(exit_field, "exit_field", torch.complex64)
    ny, nx = exit_field.shape
    _need(sources, "sources", torch.int32)
    if sources.dim() != 2 or sources.shape[1] != 2:
        raise ValueError("sources must be [n_src][2]")
    n_src = sources.shape[0]
    out = torch.empty((n_src, planes, crop, crop), dtype=torch.float32, device=exit_field.device)
    need = lib().bpm_psf_readout_workspace_size(nx, ny, planes)
    if ws is None:
        ws = workspace(need, exit_field.device)
    rc = lib().bpm_psf_readout(_ptr(exit_field), nx, ny, float(dx), float(dz), float(wavelength),
                               float(n0), float(na), int(back_steps), _ptr(sources), n_src,
                               planes, crop, float(scale), _ptr(out), _ptr(ws), ws.numel(),
                               _stream_ptr(stream))
    check(rc, "bpm_psf_readout")
    return out


def point_sources(positions: torch.Tensor, nx: int, ny: int, dx: float, wavelength: float,
                  n0: float, na: float, z_d: float = 0.0, phases: torch.Tensor | None = None,
                  out: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None):
    """Multiplexed point-source field complex64 [ny][nx] (bpm_point_sources).

    ``positions``: int32 [n][2] (y, x) on the device; ``phases``: float32 [n] or None."""
    _need(positions, "positions", torch.int32)
    if positions.dim() != 2 or positions.shape[1] != 2:
        raise ValueError("positions must be [n][2]")
    n = positions.shape[0]
    if phases is not None:
        _need(phases, "phases", torch.float32, (n,))
    dev = positions.device
    if out is None:
        out = torch.empty((ny, nx), dtype=torch.complex64, device=dev)
    _need(out, "out", torch.complex64, (ny, nx))
    need = lib().bpm_point_sources_workspace_size(nx, ny)
    if need == 0:
        raise _lib.BpmError(_lib.BPM_ERR_UNSUPPORTED_SIZE, f"nx={nx} ny={ny}")
    if ws is None:
        ws = workspace(need, dev)
    rc = lib().bpm_point_sources(_ptr(positions), _ptr(phases), n, nx, ny, float(dx),
                                 float(wavelength), float(n0), float(na), float(z_d), _ptr(out),
                                 _ptr(ws), ws.numel(), _stream_ptr(stream))
    check(rc, "bpm_point_sources")
    return out
