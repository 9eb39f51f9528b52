"""ctypes loader of libbpm.so and the declarations of include/bpm.h and
include/psf_surrogate.h.

The library is the product path: when it is missing this module raises, and
nothing falls back to another implementation.
"""
from __future__ import annotations

import atexit
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbpm.so")

BPM_OK = 0
BPM_ERR_INVALID_ARG = -1
BPM_ERR_UNSUPPORTED_SIZE = -2
BPM_ERR_WORKSPACE = -3
BPM_ERR_DEVICE = -4
BPM_ERR_NOT_FINITE = -5
BPM_WS_FORWARD = 0
BPM_WS_ADJOINT = 1

# every symbol the headers under include/ declare
EXPORTS = (
    "bpm_workspace_size", "bpm_propagate", "bpm_batch_workspace_size",
    "bpm_propagate_batch", "bpm_batch_upload", "bpm_batch_launch",
    "bpm_adjoint_workspace_size", "bpm_adjoint",
    "bpm_adjoint_batch_workspace_size", "bpm_adjoint_batch",
    "psf_surrogate_infer", "bpm_error_string", "bpm_last_error",
    "bpm_fft2_workspace_size", "bpm_fft2", "bpm_pupil_spectrum", "bpm_pupil_phase_grad",
    "bpm_psf_readout_workspace_size", "bpm_psf_readout",
    "psf_surrogate_param_count", "psf_surrogate_weights_bytes", "psf_surrogate_state_bytes",
    "psf_surrogate_workspace_size", "psf_surrogate_train_init", "psf_surrogate_train_step",
    "psf_surrogate_gradients", "psf_surrogate_params", "psf_surrogate_export",
    "psf_conv_workspace_size", "psf_conv_forward", "psf_conv_backward",
    "psf_surrogate_layer_geometry", "psf_extract_patches",
    "bpm_point_sources_workspace_size", "bpm_point_sources",
    "bpm_workspace_status", "bpm_decode_status", "bpm_set_wait_limit",
    "bpm_march_phase_times", "bpm_release",
    "bpm_propagate_noalloc", "bpm_noalloc_scratch_bytes",
    "bpm_march_variant", "bpm_march_variant_eligible", "bpm_set_march_variant",
    "bpm_propagate_adapted", "bpm_slice_means",
    "bpm_guide_star_phase", "bpm_adam_step",
    "bpm_pupil_fields_workspace_size", "bpm_pupil_fields", "bpm_zernike_workspace_size",
    "bpm_zernike_fit", "bpm_camera_accumulate",
)
BPM_MARCH_AUTO = 0
BPM_MARCH_ONE_PER_CU = 1
BPM_MARCH_TWO_PER_CU = 2
BPM_MARCH_TILED_PAIR = 3
BPM_MARCH_SMALL_BLOCKS = 4
PHASE_TIMER_WORDS = 8 + 8 * 4096
BPM_MAX_LOCKSTEP_FIELDS = 8


class BpmError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(message)
        self.code = code


class Job(ctypes.Structure):
    """Mirror of ``bpm_job``."""
    _fields_ = [("field_in", ctypes.c_void_p), ("dn", ctypes.c_void_p),
                ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("steps", ctypes.c_int),
                ("dx", ctypes.c_double), ("dz", ctypes.c_double),
                ("wavelength", ctypes.c_double), ("n0", ctypes.c_double),
                ("field_out", ctypes.c_void_p), ("intensity_out", ctypes.c_void_p),
                ("clear_steps", ctypes.c_int)]


class AdjointJob(ctypes.Structure):
    """Mirror of ``bpm_adjoint_job``."""
    _fields_ = [("field_in", ctypes.c_void_p), ("dn", ctypes.c_void_p),
                ("grad_field_out", ctypes.c_void_p), ("grad_intensity", ctypes.c_void_p),
                ("grad_field_in", ctypes.c_void_p), ("grad_spectrum_in", ctypes.c_void_p),
                ("grad_dn", ctypes.c_void_p)]


_lib = None
_V, _I, _D, _Z, _S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_char_p
_F = ctypes.c_float


def _declare(L):
    L.bpm_workspace_size.argtypes = [_I, _I, _I, _I]
    L.bpm_workspace_size.restype = _Z
    L.bpm_propagate.argtypes = [_V, _V, _I, _I, _I, _D, _D, _D, _D, _V, _V, _V, _Z, _V]
    L.bpm_propagate.restype = _I
    L.bpm_batch_workspace_size.argtypes = [ctypes.POINTER(Job), _I]
    L.bpm_batch_workspace_size.restype = _Z
    L.bpm_propagate_batch.argtypes = [ctypes.POINTER(Job), _I, _V, _Z, _V]
    L.bpm_propagate_batch.restype = _I
    for name in ("bpm_batch_upload", "bpm_batch_launch"):
        getattr(L, name).argtypes = [ctypes.POINTER(Job), _I, _V, _Z, _V]
        getattr(L, name).restype = _I
    L.bpm_adjoint_workspace_size.argtypes = [_I, _I, _I, _I]
    L.bpm_adjoint_workspace_size.restype = _Z
    L.bpm_adjoint.argtypes = [_V, _V, _I, _I, _I, _D, _D, _D, _D, _V, _V, _V, _V, _V, _I,
                              _V, _Z, _V]
    L.bpm_adjoint.restype = _I
    L.bpm_adjoint_batch_workspace_size.argtypes = [_I, _I, _I, _I, _I]
    L.bpm_adjoint_batch_workspace_size.restype = _Z
    L.bpm_adjoint_batch.argtypes = [ctypes.POINTER(AdjointJob), _I, _I, _I, _I, _D, _D, _D, _D,
                                    _I, _V, _Z, _V]
    L.bpm_adjoint_batch.restype = _I
    L.psf_surrogate_infer.argtypes = [_V, _Z, _V, _V, _I, _V, _V, _V, _Z, _V]
    L.psf_surrogate_infer.restype = _I
    for name in ("psf_surrogate_param_count", "psf_surrogate_weights_bytes",
                 "psf_surrogate_state_bytes"):
        getattr(L, name).argtypes = []
        getattr(L, name).restype = _Z
    L.psf_surrogate_workspace_size.argtypes = [_I, _I]
    L.psf_surrogate_workspace_size.restype = _Z
    L.psf_surrogate_train_init.argtypes = [_V, _V, _V]
    L.psf_surrogate_train_init.restype = _I
    L.psf_surrogate_train_step.argtypes = [_V, _V, _V, _V, _I, _F, _F, _I, _V, _V, _V, _Z, _V]
    L.psf_surrogate_train_step.restype = _I
    for name in ("psf_surrogate_gradients", "psf_surrogate_params", "psf_surrogate_export"):
        getattr(L, name).argtypes = [_V, _V, _V]
        getattr(L, name).restype = _I
    L.psf_extract_patches.argtypes = [_V, _I, _I, _I, _I, _V, _I, _V, _V]
    L.psf_extract_patches.restype = _I
    L.bpm_point_sources_workspace_size.argtypes = [_I, _I]
    L.bpm_point_sources_workspace_size.restype = _Z
    L.bpm_point_sources.argtypes = [_V, _V, _I, _I, _I, _D, _D, _D, _D, _D, _V, _V, _Z, _V]
    L.bpm_point_sources.restype = _I
    L.psf_surrogate_layer_geometry.argtypes = [_I, _V]
    L.psf_surrogate_layer_geometry.restype = _I
    L.psf_conv_workspace_size.argtypes = [_V]
    L.psf_conv_workspace_size.restype = _Z
    L.psf_conv_forward.argtypes = [_V, _V, _V, _V, _I, _V, _V, _V, _V, _Z, _V]
    L.psf_conv_forward.restype = _I
    L.psf_conv_backward.argtypes = [_V, _V, _V, _V, _V, _V, _V, _V, _V, _Z, _V]
    L.psf_conv_backward.restype = _I
    L.bpm_fft2_workspace_size.argtypes = [_I, _I]
    L.bpm_fft2_workspace_size.restype = _Z
    L.bpm_fft2.argtypes = [_V, _V, _I, _I, _I, _V, _Z, _V]
    L.bpm_fft2.restype = _I
    L.bpm_pupil_spectrum.argtypes = [_V, _V, _I, _I, _D, _D, _D, _D, _V, _V]
    L.bpm_pupil_spectrum.restype = _I
    L.bpm_pupil_phase_grad.argtypes = [_V, _V, _I, _I, _V, _V]
    L.bpm_pupil_phase_grad.restype = _I
    L.bpm_guide_star_phase.argtypes = [_V, _I, _I, _D, _D, _D, _D, _D, _D, _V, _V]
    L.bpm_guide_star_phase.restype = _I
    L.bpm_adam_step.argtypes = [_V, _V, _V, _V, ctypes.c_long, ctypes.c_float, _I, _V]
    L.bpm_adam_step.restype = _I
    L.bpm_pupil_fields_workspace_size.argtypes = [_I, _I]
    L.bpm_pupil_fields_workspace_size.restype = _Z
    L.bpm_pupil_fields.argtypes = [_V, _I, _I, _D, _D, _D, _D, _D, _I, _V, _I, _I, _V, _V, _Z, _V]
    L.bpm_pupil_fields.restype = _I
    L.bpm_zernike_workspace_size.argtypes = [_I, _I]
    L.bpm_zernike_workspace_size.restype = _Z
    L.bpm_zernike_fit.argtypes = [_V, _I, _I, _D, _D, _D, _I, _V, _V, _V, _Z, _V]
    L.bpm_zernike_fit.restype = _I
    L.bpm_camera_accumulate.argtypes = [_V, _V, _V, _I, _I, _I, _I, _V, _V]
    L.bpm_camera_accumulate.restype = _I
    L.bpm_psf_readout_workspace_size.argtypes = [_I, _I, _I]
    L.bpm_psf_readout_workspace_size.restype = _Z
    L.bpm_psf_readout.argtypes = [_V, _I, _I, _D, _D, _D, _D, _D, _I, _V, _I, _I, _I, _D, _V,
                                  _V, _Z, _V]
    L.bpm_psf_readout.restype = _I
    L.bpm_propagate_adapted.argtypes = [_V, _V, _V, _I, _I, _I, _D, _D, _D, _D, _V, _V, _V, _Z,
                                        _V]
    L.bpm_propagate_adapted.restype = _I
    L.bpm_slice_means.argtypes = [_V, _I, _I, _I, _V, _V]
    L.bpm_slice_means.restype = _I
    L.bpm_march_variant.argtypes = [_I, _I, _I]
    L.bpm_march_variant.restype = _I
    L.bpm_march_variant_eligible.argtypes = [_I, _I, _I, _I]
    L.bpm_march_variant_eligible.restype = _I
    L.bpm_set_march_variant.argtypes = [_I, _I, _I, _I]
    L.bpm_set_march_variant.restype = _I
    L.bpm_propagate_noalloc.argtypes = [_V, _V, _I, _I, _I, _D, _D, _D, _D, _V, _V, _V]
    L.bpm_propagate_noalloc.restype = _I
    L.bpm_noalloc_scratch_bytes.argtypes = []
    L.bpm_noalloc_scratch_bytes.restype = _Z
    L.bpm_release.argtypes = []
    L.bpm_release.restype = None
    L.bpm_march_phase_times.argtypes = [ctypes.POINTER(Job), _I, _V, _Z, _V, _Z, _V]
    L.bpm_march_phase_times.restype = _I
    L.bpm_workspace_status.argtypes = [_V, _Z, _V]
    L.bpm_workspace_status.restype = _I
    L.bpm_decode_status.argtypes = [ctypes.c_uint]
    L.bpm_decode_status.restype = _I
    L.bpm_set_wait_limit.argtypes = [ctypes.c_ulonglong]
    L.bpm_set_wait_limit.restype = _I
    L.bpm_error_string.argtypes = [_I]
    L.bpm_error_string.restype = _S
    L.bpm_last_error.argtypes = []
    L.bpm_last_error.restype = _S


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
        # free the library's pinned staging while the HIP runtime is alive
        atexit.register(L.bpm_release)
    return _lib


def check(rc: int, name: str) -> None:
    if rc != BPM_OK:
        L = lib()
        msg = L.bpm_last_error().decode(errors="replace")
        raise BpmError(rc, f"{name}: {L.bpm_error_string(rc).decode()} ({msg})")
