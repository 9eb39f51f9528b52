"""FP64 CPU oracle of the split-step beam-propagation march (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product package.  The C
source ``oracle.c`` holds the arithmetic and states what it computes; this
module only builds it, marshals numpy arrays and upcasts inputs to float64.

Parity status of each function (what pins it, see tests/test_oracle_*.py):

* fft1d / fft2d   -- brute-force O(N^2) DFT in pure Python, inverse round trip.
* propagator      -- plane-wave closed forms (homogeneous phase, single mode),
                     lattice-point count of the propagating disc, composition.
* bpm_forward     -- dense-matrix recursion on 8x8, Parseval, thin-grating
                     Jacobi-Anger closed form, Gaussian-beam paraxial width,
                     linearity (multiplexing), resume.
* bpm_forward_adapted -- dn_ref = 0 is bpm_forward; a plane wave through
                     homogeneous layers expanded about their own index
                     follows the exact layered-medium phase; modes between
                     the n0 and the adapted evanescent cut propagate.
* bpm_adjoint     -- dot-product test, central finite differences, phase
                     conjugation optimum, per-slice gauge invariance.
* conv3d_*        -- (surrogate) direct definition vs scipy correlate and
                     central finite differences.
* psf_readout     -- free-space composition and dn = 0 focus.
* point_sources   -- one source = numpy's inverse FFT of the closed-form
                     spectrum, unit norm, shift and phase linearity.
* surrogate_net   -- (module) central finite differences of the loss.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "conv_oracle.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc -O3 -fopenmp (no fast-math)."""
    srcs = [s for s in _SRC if os.path.exists(s)]
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-Wall", "-Wno-unknown-pragmas", "-o", tmp] + srcs + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_I = ctypes.c_int
_D = ctypes.c_double


def _declare(L):
    L.oracle_fft1d.argtypes = [_dp, _I, _I]
    L.oracle_fft2d.argtypes = [_dp, _I, _I, _I]
    L.oracle_propagator.argtypes = [_I, _I, _D, _D, _D, _D, _dp]
    L.oracle_bpm_forward.argtypes = [_dp, _dp, _I, _I, _I, _D, _D, _D, _D, _dp, _dp]
    L.oracle_bpm_forward_adapted.argtypes = [_dp, _dp, _dp, _I, _I, _I, _D, _D, _D, _D, _dp,
                                             _dp]
    L.oracle_bpm_forward_adapted.restype = _I
    L.oracle_bpm_adjoint.argtypes = [_dp, _dp, _I, _I, _I, _D, _D, _D, _D,
                                     _dp, _dp, _dp, _dp, _dp]
    L.oracle_set_threads.argtypes = [_I]
    L.oracle_psf_readout.argtypes = [_dp, _I, _I, _D, _D, _D, _D, _D, _I,
                                     ctypes.POINTER(ctypes.c_int), _I, _I, _I, _D, _dp]
    L.oracle_psf_readout.restype = _I
    L.oracle_point_sources.argtypes = [ctypes.POINTER(ctypes.c_int), _dp, _I, _I, _I, _D, _D, _D,
                                       _D, _D, _dp]
    L.oracle_point_sources.restype = _I
    for name in ("oracle_set_threads", "oracle_fft1d", "oracle_fft2d", "oracle_propagator",
                 "oracle_bpm_forward", "oracle_bpm_adjoint"):
        getattr(L, name).restype = _I
    if hasattr(L, "oracle_conv3d_forward"):
        _declare_conv(L)


def _declare_conv(L):
    # forward(x, w, b, y, N, Ci, D, H, W, Co, kd, kh, kw, sd, sh, sw, pd, ph, pw, relu)
    # backward(x, w, dy, dx, dw, db, N, Ci, D, H, W, Co, kd, kh, kw, sd, sh, sw, pd, ph, pw)
    L.oracle_conv3d_forward.argtypes = [_dp, _dp, _dp, _dp] + [_I] * 16
    L.oracle_conv3d_backward.argtypes = [_dp] * 6 + [_I] * 15
    L.oracle_conv3d_forward.restype = _I
    L.oracle_conv3d_backward.restype = _I


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, name):
    if rc != 0:
        raise ValueError(f"{name} failed with code {rc}")


# ---------------------------------------------------------------------------
# public helpers (numpy in, numpy out; float64 / complex128)

def fft1d(x, sign=-1):
    a = _c128(x).copy()
    _check(lib().oracle_fft1d(_ptr(a.view(np.float64)), a.shape[-1], sign), "fft1d")
    return a


def fft2d(x, sign=-1):
    a = _c128(x).copy()
    ny, nx = a.shape
    _check(lib().oracle_fft2d(_ptr(a.view(np.float64)), nx, ny, sign), "fft2d")
    return a


def propagator(nx, ny, dx, dz, wavelength, n0):
    h = np.empty((ny, nx), dtype=np.complex128)
    _check(lib().oracle_propagator(nx, ny, dx, dz, wavelength, n0, _ptr(h.view(np.float64))),
           "propagator")
    return h


def bpm_forward(u0, dn, dx, dz, wavelength, n0, intensity=True):
    """March ``u0`` ([ny][nx]) through ``dn`` ([steps][ny][nx]).

    Returns (u_out complex128, I float64 [steps][ny][nx] or None)."""
    u = _c128(u0)
    d = _f64(dn)
    steps, ny, nx = d.shape
    out = np.empty_like(u)
    inten = np.empty((steps, ny, nx), dtype=np.float64) if intensity else None
    rc = lib().oracle_bpm_forward(_ptr(u.view(np.float64)), _ptr(d), nx, ny, steps,
                                  dx, dz, wavelength, n0, _ptr(out.view(np.float64)),
                                  _ptr(inten))
    _check(rc, "bpm_forward")
    return out, inten


def bpm_forward_adapted(u0, dn, dn_ref, dx, dz, wavelength, n0, intensity=True):
    """March with a per-slice reference index n0 + dn_ref[j] (the locally
    adapted expansion; see oracle.c).  Returns (u_out, I or None)."""
    u = _c128(u0)
    d = _f64(dn)
    r = _f64(dn_ref)
    steps, ny, nx = d.shape
    if r.shape != (steps,):
        raise ValueError(f"dn_ref has shape {r.shape}, expected ({steps},)")
    out = np.empty_like(u)
    inten = np.empty((steps, ny, nx), dtype=np.float64) if intensity else None
    rc = lib().oracle_bpm_forward_adapted(_ptr(u.view(np.float64)), _ptr(d), _ptr(r), nx, ny,
                                          steps, dx, dz, wavelength, n0,
                                          _ptr(out.view(np.float64)), _ptr(inten))
    _check(rc, "bpm_forward_adapted")
    return out, inten


def bpm_adjoint(u0, dn, dx, dz, wavelength, n0, grad_u_out=None, grad_intensity=None):
    """Gradients of a loss through the march (PyTorch complex convention).

    Returns (grad_u0, grad_spectrum0, grad_dn)."""
    u = _c128(u0)
    d = _f64(dn)
    steps, ny, nx = d.shape
    gu = None if grad_u_out is None else _c128(grad_u_out)
    gi = None if grad_intensity is None else _f64(grad_intensity)
    g0 = np.empty_like(u)
    s0 = np.empty_like(u)
    gdn = np.empty((steps, ny, nx), dtype=np.float64)
    rc = lib().oracle_bpm_adjoint(_ptr(u.view(np.float64)), _ptr(d), nx, ny, steps,
                                  dx, dz, wavelength, n0,
                                  None if gu is None else _ptr(gu.view(np.float64)),
                                  _ptr(gi), _ptr(g0.view(np.float64)),
                                  _ptr(s0.view(np.float64)), _ptr(gdn))
    _check(rc, "bpm_adjoint")
    return g0, s0, gdn


def psf_readout(exit_field, dx, dz, wavelength, n0, na, back_steps, sources, planes=32,
                crop=32, scale=1.0):
    """Refocused PSF stacks of a multiplexed run: [n_src][planes][crop][crop]."""
    u = _c128(exit_field)
    ny, nx = u.shape
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32).reshape(-1, 2))
    out = np.empty((len(src), planes, crop, crop), dtype=np.float64)
    rc = lib().oracle_psf_readout(_ptr(u.view(np.float64)), nx, ny, dx, dz, wavelength, n0, na,
                                  int(back_steps), src.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                  len(src), planes, crop, float(scale), _ptr(out))
    _check(rc, "psf_readout")
    return out


def _conv_geo(x_shape, w_shape, stride, pad):
    N, Ci, D, H, W = x_shape
    Co, Ci2, kd, kh, kw = w_shape
    if Ci2 != Ci:
        raise ValueError("channel mismatch")
    sd, sh, sw = stride
    pd, ph, pw = pad
    out = (N, Co, (D + 2 * pd - kd) // sd + 1, (H + 2 * ph - kh) // sh + 1,
           (W + 2 * pw - kw) // sw + 1)
    return [N, Ci, D, H, W, Co, kd, kh, kw, sd, sh, sw, pd, ph, pw], out


def conv3d_forward(x, w, b=None, stride=(1, 1, 1), pad=(1, 1, 1), relu=False):
    """Direct-loop 3-D cross-correlation (NCDHW), float64."""
    x, w = _f64(x), _f64(w)
    b = None if b is None else _f64(b)
    geo, out_shape = _conv_geo(x.shape, w.shape, stride, pad)
    y = np.empty(out_shape)
    _check(lib().oracle_conv3d_forward(_ptr(x), _ptr(w), _ptr(b), _ptr(y), *geo, int(relu)),
           "conv3d_forward")
    return y


def conv3d_backward(x, w, dy, stride=(1, 1, 1), pad=(1, 1, 1)):
    """Gradients (dx, dw, db) of the convolution for an upstream gradient dy."""
    x, w, dy = _f64(x), _f64(w), _f64(dy)
    geo, out_shape = _conv_geo(x.shape, w.shape, stride, pad)
    if dy.shape != out_shape:
        raise ValueError(f"dy has shape {dy.shape}, expected {out_shape}")
    dx, dw, db = np.empty(x.shape), np.empty(w.shape), np.empty(w.shape[0])
    _check(lib().oracle_conv3d_backward(_ptr(x), _ptr(w), _ptr(dy), _ptr(dx), _ptr(dw), _ptr(db),
                                        *geo), "conv3d_backward")
    return dx, dw, db


def point_sources(nx, ny, dx, wavelength, n0, na, z_d, positions, phases=None):
    """Multiplexed point-source field [ny][nx] (complex128): the weighted sum of
    integer circular shifts of one unit-norm NA-limited source."""
    pos = np.ascontiguousarray(np.asarray(positions, dtype=np.int32).reshape(-1, 2))
    ph = None if phases is None else _f64(phases)
    out = np.empty((ny, nx), dtype=np.complex128)
    rc = lib().oracle_point_sources(pos.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _ptr(ph),
                                    len(pos), nx, ny, dx, wavelength, n0, na, z_d,
                                    _ptr(out.view(np.float64)))
    _check(rc, "point_sources")
    return out


def set_threads(n: int = 0) -> int:
    """Thread count of the oracle's OpenMP loops (0: keep); returns the count."""
    return int(lib().oracle_set_threads(int(n)))
