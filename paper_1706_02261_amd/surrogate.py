"""Torch-facing binding of the learned PSF surrogate (include/psf_surrogate.h
and psf_surrogate_infer in include/bpm.h).  Argument marshalling only: the
network's forward, backward and optimizer steps run in libbpm.so.
"""
from __future__ import annotations

import ctypes
import math

import torch

from . import _lib
from ._lib import check, lib
from .bpm import _need, _ptr, _stream_ptr, workspace

PATCH = (64, 32, 32)       # dn patch (z, y, x)
PSF = (32, 32, 32)         # PSF stack (plane, y, x)
N_LAYERS = 6
HEAD_C = 64
IN_USED = 5                # input channels carrying data (dn, depth mask, cy, cx, r^2)


def _geom_array(geom):
    g = (ctypes.c_int * 15)(*[int(v) for v in geom])
    return g


def layer_geometry(layer: int):
    """The 15 defining integers of layer ``layer`` (N = 1)."""
    g = (ctypes.c_int * 15)()
    check(lib().psf_surrogate_layer_geometry(int(layer), g), "psf_surrogate_layer_geometry")
    return list(g)


def conv_dims(geom):
    """(Do, Ho, Wo, taps, K, Kp) of a geometry."""
    N, D, H, W, Ci, Co, kd, kh, kw, sd, sh, sw, pd, ph, pw = geom
    Do = (D + 2 * pd - kd) // sd + 1
    Ho = (H + 2 * ph - kh) // sh + 1
    Wo = (W + 2 * pw - kw) // sw + 1
    taps = kd * kh * kw
    K = taps * Ci
    return Do, Ho, Wo, taps, K, (K + 15) // 16 * 16


def param_count() -> int:
    return int(lib().psf_surrogate_param_count())


def param_slices():
    """Slices of the flat parameter vector: ('w', l), ('b', l), 'we', 'be'."""
    out, o = {}, 0
    geoms = [layer_geometry(l) for l in range(N_LAYERS)]
    for l, g in enumerate(geoms):
        n = g[5] * conv_dims(g)[5]
        out[("w", l)] = slice(o, o + n)
        o += n
    for l, g in enumerate(geoms):
        out[("b", l)] = slice(o, o + g[5])
        o += g[5]
    out["we"] = slice(o, o + HEAD_C)
    o += HEAD_C
    out["be"] = slice(o, o + 1)
    o += 1
    assert o == param_count()
    return out


def init_params(seed: int = 0, out_bias: float = -4.5, hidden_bias: float = 0.05) -> torch.Tensor:
    """He-normal conv weights (zero K padding), small positive biases of the
    ReLU layers (``hidden_bias``, keeps units alive early in training), the PSF
    layer's bias ``out_bias`` (softplus(-4.5) ~ 0.011, the order of a PSF
    stack's mean), small head weights; float32 on the CPU."""
    gen = torch.Generator().manual_seed(seed)
    p = torch.zeros(param_count(), dtype=torch.float32)
    sl = param_slices()
    for l in range(N_LAYERS):
        g = layer_geometry(l)
        Co = g[5]
        _, _, _, taps, K, Kp = conv_dims(g)
        fan_in = taps * (IN_USED if l == 0 else g[4])
        w = torch.zeros(Co, Kp)
        wk = torch.randn(Co, taps, g[4], generator=gen) * math.sqrt(2.0 / fan_in)
        if l == 0:  # channels IN_USED.. of the 8-channel input are zero padding
            wk[:, :, IN_USED:] = 0.0
        w[:, :K] = wk.reshape(Co, K)
        p[sl[("w", l)]] = w.reshape(-1)
        p[sl[("b", l)]] = hidden_bias
    p[sl[("b", N_LAYERS - 1)]] = out_bias
    p[sl["we"]] = torch.randn(HEAD_C, generator=gen) * 0.01
    p[sl["be"]] = -3.0
    return p


# ---------------------------------------------------------------------------
# building blocks (used by the parity tests)

def conv_forward(x: torch.Tensor, w: torch.Tensor, bias: torch.Tensor, geom, epilogue: int = 0,
                 stream=None):
    """One convolution: x bf16 [N][D][H][W][Ci], w fp32 [Co][Kp], bias fp32 [Co].

    epilogue 0 -> bf16 ReLU output [N][Do][Ho][Wo][Co];
    epilogue 1 -> (softplus output, pre-activation), fp32 [N][Co][Ho][Wo]."""
    N, D, H, W, Ci, Co = geom[:6]
    Do, Ho, Wo, _, _, Kp = conv_dims(geom)
    _need(x, "x", torch.bfloat16, (N, D, H, W, Ci))
    _need(w, "w", torch.float32, (Co, Kp))
    _need(bias, "bias", torch.float32, (Co,))
    dev = x.device
    g = _geom_array(geom)
    ws = workspace(max(int(lib().psf_conv_workspace_size(g)), 256), dev)
    if epilogue == 0:
        y = torch.empty((N, Do, Ho, Wo, Co), dtype=torch.bfloat16, device=dev)
        rc = lib().psf_conv_forward(_ptr(x), _ptr(w), _ptr(bias), g, 0, _ptr(y), None, None,
                                    _ptr(ws), ws.numel(), _stream_ptr(stream))
        check(rc, "psf_conv_forward")
        return y
    yf = torch.empty((N, Co, Ho, Wo), dtype=torch.float32, device=dev)
    z = torch.empty_like(yf)
    rc = lib().psf_conv_forward(_ptr(x), _ptr(w), _ptr(bias), g, int(epilogue), None, _ptr(yf),
                                _ptr(z), _ptr(ws), ws.numel(), _stream_ptr(stream))
    check(rc, "psf_conv_forward")
    return yf, z


def conv_backward(x: torch.Tensor, w: torch.Tensor, dy: torch.Tensor, geom,
                  xmask: torch.Tensor | None = None, want_dx: bool = True,
                  want_dw: bool = True, stream=None):
    """Gradients of one convolution: returns (dx bf16, dw fp32 [Co][Kp], db fp32 [Co])."""
    N, D, H, W, Ci, Co = geom[:6]
    Do, Ho, Wo, _, _, Kp = conv_dims(geom)
    _need(x, "x", torch.bfloat16, (N, D, H, W, Ci))
    _need(w, "w", torch.float32, (Co, Kp))
    _need(dy, "dy", torch.bfloat16, (N, Do, Ho, Wo, Co))
    if xmask is not None:
        _need(xmask, "xmask", torch.bfloat16, (N, D, H, W, Ci))
    dev = x.device
    g = _geom_array(geom)
    dx = torch.empty_like(x) if want_dx else None
    dw = torch.empty((Co, Kp), dtype=torch.float32, device=dev) if want_dw else None
    db = torch.empty(Co, dtype=torch.float32, device=dev) if want_dw else None
    ws = workspace(max(int(lib().psf_conv_workspace_size(g)), 256), dev)
    rc = lib().psf_conv_backward(_ptr(x), _ptr(w), _ptr(dy), _ptr(xmask), g, _ptr(dx), _ptr(dw),
                                 _ptr(db), _ptr(ws), ws.numel(), _stream_ptr(stream))
    check(rc, "psf_conv_backward")
    return dx, dw, db


# ---------------------------------------------------------------------------
# the network

def extract_patches(dn: torch.Tensor, sources: torch.Tensor, z0: int = 0,
                    out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """[n][64][32][32] windows of dn [nz][ny][nx] around sources (int32 [n][2] (y, x))."""
    _need(dn, "dn", torch.float32)
    if dn.dim() != 3:
        raise ValueError("dn must be [nz][ny][nx]")
    _need(sources, "sources", torch.int32)
    if sources.dim() != 2 or sources.shape[1] != 2:
        raise ValueError("sources must be [n][2]")
    n = sources.shape[0]
    if out is None:
        out = torch.empty((n,) + PATCH, dtype=torch.float32, device=dn.device)
    _need(out, "out", torch.float32, (n,) + PATCH)
    nz, ny, nx = dn.shape
    rc = lib().psf_extract_patches(_ptr(dn), nz, ny, nx, int(z0), _ptr(sources), n, _ptr(out),
                                   _stream_ptr(stream))
    check(rc, "psf_extract_patches")
    return out


def weights_bytes() -> int:
    return int(lib().psf_surrogate_weights_bytes())


def infer(weights: torch.Tensor, dn_patches: torch.Tensor, depth: torch.Tensor,
          psf_out: torch.Tensor | None = None, pred_err: torch.Tensor | None = None,
          ws: torch.Tensor | None = None, stream=None):
    """PSF stacks [B][32][32][32] and predicted relative errors [B]."""
    _need(weights, "weights", torch.uint8, (weights_bytes(),))
    _need(dn_patches, "dn_patches", torch.float32)
    B = dn_patches.shape[0]
    if tuple(dn_patches.shape[1:]) != PATCH:
        raise ValueError(f"dn_patches must be [B]{list(PATCH)}")
    _need(depth, "depth", torch.float32, (B,))
    dev = dn_patches.device
    if psf_out is None:
        psf_out = torch.empty((B,) + PSF, dtype=torch.float32, device=dev)
    if pred_err is None:
        pred_err = torch.empty(B, dtype=torch.float32, device=dev)
    _need(psf_out, "psf_out", torch.float32, (B,) + PSF)
    _need(pred_err, "pred_err", torch.float32, (B,))
    if ws is None:
        ws = workspace(max(int(lib().psf_surrogate_workspace_size(B, 0)), 256), dev)
    rc = lib().psf_surrogate_infer(_ptr(weights), weights.numel(), _ptr(dn_patches), _ptr(depth),
                                   B, _ptr(psf_out), _ptr(pred_err), _ptr(ws), ws.numel(),
                                   _stream_ptr(stream))
    check(rc, "psf_surrogate_infer")
    return psf_out, pred_err


class PSFSurrogate:
    """Training state of the surrogate on one device (Adam, step counter)."""

    def __init__(self, device, params: torch.Tensor | None = None, seed: int = 0, stream=None):
        self.device = torch.device(device)
        if params is None:
            params = init_params(seed)
        params = params.to(self.device, torch.float32).contiguous()
        _need(params, "params", torch.float32, (param_count(),))
        self.state = workspace(int(lib().psf_surrogate_state_bytes()), self.device)
        self.step_count = 0
        self._ws = None
        self.loss = torch.zeros(2, dtype=torch.float32, device=self.device)
        rc = lib().psf_surrogate_train_init(_ptr(self.state), _ptr(params), _stream_ptr(stream))
        check(rc, "psf_surrogate_train_init")

    def _workspace(self, B: int):
        need = max(int(lib().psf_surrogate_workspace_size(B, 1)), 256)
        if self._ws is None or self._ws.numel() < need:
            self._ws = workspace(need, self.device)
        return self._ws

    def train_step(self, dn_patches, depth, target, lr: float, err_weight: float = 1.0,
                   err_true: torch.Tensor | None = None, stream=None):
        """One step; returns the device tensor [psf loss, error-head loss].  With
        lr = 0 only the gradients are computed (no update, no step count)."""
        _need(dn_patches, "dn_patches", torch.float32)
        B = dn_patches.shape[0]
        if tuple(dn_patches.shape[1:]) != PATCH:
            raise ValueError(f"dn_patches must be [B]{list(PATCH)}")
        _need(depth, "depth", torch.float32, (B,))
        _need(target, "target", torch.float32, (B,) + PSF)
        if err_true is not None:
            _need(err_true, "err_true", torch.float32, (B,))
        ws = self._workspace(B)
        step = self.step_count + 1 if lr > 0 else 0
        rc = lib().psf_surrogate_train_step(_ptr(self.state), _ptr(dn_patches), _ptr(depth),
                                            _ptr(target), B, float(lr), float(err_weight), step,
                                            _ptr(self.loss), _ptr(err_true), _ptr(ws), ws.numel(),
                                            _stream_ptr(stream))
        check(rc, "psf_surrogate_train_step")
        if lr > 0:
            self.step_count += 1
        return self.loss

    def fit(self, dn_patches, depth, target, seconds: float | None = None,
            epochs: int | None = None, batch: int = 64, lr: float = 5e-4,
            err_weight: float = 1.0, seed: int = 0, warmup_steps: int = 1000,
            log=None) -> int:
        """Adam over shuffled mini-batches until ``epochs`` epochs or ``seconds``
        of wall time have passed (whichever is given; both: the first reached).
        The learning rate rises linearly over the first ``warmup_steps`` steps
        and then decays as lr / (1 + 0.05 e), e = epochs since the warm-up.  A
        short warm-up to a large rate drives the softplus output of the PSF
        layer to zero everywhere within a few hundred steps (loss 1, vanishing
        gradient), a state training leaves only after tens of epochs.  Returns
        the number of epochs run."""
        import time
        if seconds is None and epochs is None:
            raise ValueError("give seconds or epochs")
        n = dn_patches.shape[0]
        nb = n // batch
        if nb < 1:
            raise ValueError(f"{n} samples are fewer than one batch of {batch}")
        order = torch.Generator().manual_seed(seed)
        t0 = time.perf_counter()
        epoch = 0
        k = 0
        warm = max(1, warmup_steps)
        while ((epochs is None or epoch < epochs) and
               (seconds is None or time.perf_counter() - t0 < seconds)):
            perm = torch.randperm(n, generator=order).to(self.device)
            total = torch.zeros(2, dtype=torch.float32, device=self.device)
            for b in range(nb):
                i = perm[b * batch:(b + 1) * batch]
                rate = lr * min(1.0, (k + 1) / warm) / (1.0 + 0.05 * max(0, k + 1 - warm) / nb)
                total += self.train_step(dn_patches[i].contiguous(), depth[i].contiguous(),
                                         target[i].contiguous(), lr=rate, err_weight=err_weight)
                k += 1
            torch.cuda.synchronize(self.device)
            epoch += 1
            if log is not None:
                log(epoch, (total / nb).tolist(), time.perf_counter() - t0)
        return epoch

    def gradients(self, stream=None) -> torch.Tensor:
        g = torch.empty(param_count(), dtype=torch.float32, device=self.device)
        check(lib().psf_surrogate_gradients(_ptr(self.state), _ptr(g), _stream_ptr(stream)),
              "psf_surrogate_gradients")
        return g

    def params(self, stream=None) -> torch.Tensor:
        p = torch.empty(param_count(), dtype=torch.float32, device=self.device)
        check(lib().psf_surrogate_params(_ptr(self.state), _ptr(p), _stream_ptr(stream)),
              "psf_surrogate_params")
        return p

    def export(self, stream=None) -> torch.Tensor:
        blob = workspace(weights_bytes(), self.device)
        check(lib().psf_surrogate_export(_ptr(self.state), _ptr(blob), _stream_ptr(stream)),
              "psf_surrogate_export")
        return blob
