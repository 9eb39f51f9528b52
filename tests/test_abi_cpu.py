"""C-ABI contract checks that need no GPU.

The library loads on a host without a GPU, exports every function that the
headers under include/ declare, and rejects bad arguments on the host before any HIP
call is made.  Pointers here are host addresses used only as non-null,
aligned placeholders: every call below fails validation first.
"""
import ctypes
import glob
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


@pytest.fixture(scope="module")
def L():
    from paper_1706_02261_amd import _lib
    return _lib.lib()


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(\w+)\s*\(", text, flags=re.M))
    return sorted(names)


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert "bpm_propagate" in names and "bpm_adjoint" in names and len(names) >= 13
    for n in names:
        assert hasattr(L, n), n


def test_binding_lists_every_export():
    from paper_1706_02261_amd import _lib
    assert set(declared_functions()) == set(_lib.EXPORTS)


def test_error_strings(L):
    for code in (0, -1, -2, -3, -4, -5):
        assert L.bpm_error_string(code)
    assert L.bpm_error_string(-99) == b"unknown error code"


@pytest.mark.parametrize("nx,ny", [(16, 64), (64, 4096), (100, 128), (0, 64), (-64, 64)])
def test_workspace_size_rejects_unsupported_sizes(L, nx, ny):
    assert L.bpm_workspace_size(nx, ny, 8, 0) == 0


def test_workspace_sizes(L):
    fwd = L.bpm_workspace_size(1024, 1024, 1024, 0)
    assert fwd >= 8 * 1024 * 1024                      # the propagator table
    adj = L.bpm_adjoint_workspace_size(256, 256, 512, 0)
    k = math.ceil(math.sqrt(512))
    fields = math.ceil(512 / k) + 2 * k + 2            # checkpoints, two segment buffers
    assert adj >= fields * 256 * 256 * 8
    assert L.bpm_workspace_size(256, 256, 512, 1) == adj
    assert L.bpm_adjoint_workspace_size(256, 256, 512, 513) == 0
    assert L.bpm_adjoint_workspace_size(256, 256, 512, 1) > adj


class Buf:
    """Host placeholder memory, aligned, never dereferenced by these calls."""

    def __init__(self, n=4096):
        self.a = np.zeros(n + 64, np.uint8)
        base = self.a.ctypes.data
        self.p = base + (-base) % 256

    def __int__(self):
        return self.p


def call_propagate(L, nx=64, ny=64, steps=2, dx=0.2, dz=0.2, lam=0.5, n0=1.33,
                   fin=True, dn=True, fout=True, ws_bytes=None):
    b = Buf()
    ws = b.p if ws_bytes != -1 else None
    wsb = L.bpm_workspace_size(64, 64, 2, 0) if ws_bytes is None else max(ws_bytes, 0)
    return L.bpm_propagate(b.p if fin else None, b.p if dn else None, nx, ny, steps, dx, dz, lam,
                           n0, b.p if fout else None, None, ws, wsb, None)


def test_propagate_validation(L):
    from paper_1706_02261_amd import _lib as B
    assert call_propagate(L, nx=100) == B.BPM_ERR_UNSUPPORTED_SIZE
    assert call_propagate(L, ny=4096) == B.BPM_ERR_UNSUPPORTED_SIZE
    assert call_propagate(L, steps=-1) == B.BPM_ERR_INVALID_ARG
    assert call_propagate(L, dx=float("nan")) == B.BPM_ERR_NOT_FINITE
    assert call_propagate(L, dz=float("inf")) == B.BPM_ERR_NOT_FINITE
    assert call_propagate(L, lam=0.0) == B.BPM_ERR_NOT_FINITE
    assert call_propagate(L, n0=-1.0) == B.BPM_ERR_NOT_FINITE
    assert call_propagate(L, fin=False) == B.BPM_ERR_INVALID_ARG
    assert call_propagate(L, fout=False) == B.BPM_ERR_INVALID_ARG
    assert call_propagate(L, dn=False) == B.BPM_ERR_INVALID_ARG
    assert call_propagate(L, ws_bytes=16) == B.BPM_ERR_WORKSPACE
    assert call_propagate(L, ws_bytes=-1) == B.BPM_ERR_WORKSPACE
    assert b"workspace" in L.bpm_last_error()


def test_adjoint_validation(L):
    from paper_1706_02261_amd import _lib as B
    b = Buf()
    ws = L.bpm_adjoint_workspace_size(64, 64, 4, 0)
    rc = L.bpm_adjoint(b.p, b.p, 64, 64, 4, 0.2, 0.2, 0.5, 1.33, None, None, b.p, None, None,
                       5, b.p, ws, None)
    assert rc == B.BPM_ERR_INVALID_ARG and b"checkpoint_every" in L.bpm_last_error()
    # field_in may be NULL only for the linear adjoint (no intensity or dn gradient)
    rc = L.bpm_adjoint(None, b.p, 64, 64, 4, 0.2, 0.2, 0.5, 1.33, None, None, b.p, None, b.p,
                       0, b.p, ws, None)
    assert rc == B.BPM_ERR_INVALID_ARG and b"field_in" in L.bpm_last_error()
    rc = L.bpm_adjoint(None, b.p, 64, 64, 4, 0.2, 0.2, 0.5, 1.33, b.p, b.p, b.p, None, None,
                       0, b.p, ws, None)
    assert rc == B.BPM_ERR_INVALID_ARG and b"field_in" in L.bpm_last_error()
    rc = L.bpm_adjoint(b.p, b.p, 64, 64, 4, 0.2, 0.2, 0.5, 1.33, None, None, b.p, None, None,
                       0, b.p, 100, None)
    assert rc == B.BPM_ERR_WORKSPACE


def test_adjoint_batch_validation(L):
    from paper_1706_02261_amd import _lib as B
    b = Buf()
    one = L.bpm_adjoint_workspace_size(64, 64, 4, 0)
    plan = L.bpm_fft2_workspace_size(64, 64)
    # the plan once, then each field's checkpoints and work fields
    assert L.bpm_adjoint_batch_workspace_size(1, 64, 64, 4, 0) == one
    assert L.bpm_adjoint_batch_workspace_size(3, 64, 64, 4, 0) == plan + 3 * (one - plan)
    assert L.bpm_adjoint_batch_workspace_size(0, 64, 64, 4, 0) == 0
    assert L.bpm_adjoint_batch_workspace_size(9, 64, 64, 4, 0) == 0
    assert L.bpm_adjoint_batch_workspace_size(2, 100, 64, 4, 0) == 0
    jobs = (B.AdjointJob * 2)()
    for k in range(2):
        jobs[k] = B.AdjointJob(b.p, b.p, None, None, b.p, None, None)
    ws = L.bpm_adjoint_batch_workspace_size(2, 64, 64, 4, 0)
    for n in (0, 9):
        rc = L.bpm_adjoint_batch(jobs, n, 64, 64, 4, 0.2, 0.2, 0.5, 1.33, 0, b.p, ws, None)
        assert rc == B.BPM_ERR_INVALID_ARG and b"n_fields" in L.bpm_last_error()
    rc = L.bpm_adjoint_batch(None, 2, 64, 64, 4, 0.2, 0.2, 0.5, 1.33, 0, b.p, ws, None)
    assert rc == B.BPM_ERR_INVALID_ARG
    rc = L.bpm_adjoint_batch(jobs, 2, 64, 64, 4, 0.2, 0.2, 0.5, 1.33, 0, b.p, ws - 1, None)
    assert rc == B.BPM_ERR_WORKSPACE
    # the second job asks for dn gradients without its forward field
    jobs[1] = B.AdjointJob(None, b.p, b.p, None, b.p, None, b.p)
    rc = L.bpm_adjoint_batch(jobs, 2, 64, 64, 4, 0.2, 0.2, 0.5, 1.33, 0, b.p, ws, None)
    assert rc == B.BPM_ERR_INVALID_ARG and b"job 1" in L.bpm_last_error()
    jobs[1] = B.AdjointJob(b.p, None, None, None, b.p, None, None)
    rc = L.bpm_adjoint_batch(jobs, 2, 64, 64, 4, 0.2, 0.2, 0.5, 1.33, 0, b.p, ws, None)
    assert rc == B.BPM_ERR_INVALID_ARG and b"dn" in L.bpm_last_error()
    rc = L.bpm_adjoint_batch(jobs, 2, 64, 64, 4, 0.2, 0.2, 0.5, 1.33, 5, b.p, ws, None)
    assert rc == B.BPM_ERR_INVALID_ARG and b"checkpoint_every" in L.bpm_last_error()


def test_batch_validation(L):
    from paper_1706_02261_amd import _lib as B
    b = Buf()
    jobs = (B.Job * 2)()
    jobs[0] = B.Job(b.p, b.p, 64, 64, 3, 0.2, 0.2, 0.5, 1.33, b.p, 0)
    jobs[1] = B.Job(b.p, b.p, 48, 64, 3, 0.2, 0.2, 0.5, 1.33, b.p, 0)
    assert L.bpm_batch_workspace_size(jobs, 2) == 0
    assert L.bpm_propagate_batch(jobs, 2, b.p, 1 << 30, None) == B.BPM_ERR_UNSUPPORTED_SIZE
    assert b"job 1" in L.bpm_last_error()
    assert L.bpm_propagate_batch(jobs, 0, b.p, 1 << 30, None) == B.BPM_ERR_INVALID_ARG
    jobs[1] = B.Job(b.p, None, 64, 64, 3, 0.2, 0.2, 0.5, 1.33, b.p, 0)
    assert L.bpm_propagate_batch(jobs, 2, b.p, 1 << 30, None) == B.BPM_ERR_INVALID_ARG
    jobs[1] = B.Job(b.p, b.p, 64, 64, 3, 0.2, 0.2, 0.5, 1.33, b.p, 0, 4)     # clear_steps > steps
    assert L.bpm_propagate_batch(jobs, 2, b.p, 1 << 30, None) == B.BPM_ERR_INVALID_ARG
    assert b"clear_steps" in L.bpm_last_error()
    jobs[1] = B.Job(b.p, b.p, 64, 64, 3, 0.2, 0.2, 0.5, 1.33, b.p, 0, -1)
    assert L.bpm_propagate_batch(jobs, 2, b.p, 1 << 30, None) == B.BPM_ERR_INVALID_ARG
    jobs[1] = B.Job(b.p, b.p, 64, 64, 3, 0.2, 0.2, 0.5, 1.33, b.p, 0)
    need = L.bpm_batch_workspace_size(jobs, 2)
    assert need > 2 * L.bpm_workspace_size(64, 64, 3, 0)
    assert L.bpm_propagate_batch(jobs, 2, b.p, need - 1, None) == B.BPM_ERR_WORKSPACE
    # the two halves validate like the whole call (no device work on a bad argument)
    for half in (L.bpm_batch_upload, L.bpm_batch_launch):
        assert half(jobs, 2, b.p, need - 1, None) == B.BPM_ERR_WORKSPACE
        assert half(jobs, 0, b.p, need, None) == B.BPM_ERR_INVALID_ARG
        bad = (B.Job * 2)(jobs[0], B.Job(b.p, None, 64, 64, 3, 0.2, 0.2, 0.5, 1.33, b.p, 0))
        assert half(bad, 2, b.p, need, None) == B.BPM_ERR_INVALID_ARG
        assert b"job 1" in L.bpm_last_error()


def test_helper_validation(L):
    from paper_1706_02261_amd import _lib as B
    b = Buf()
    assert L.bpm_fft2(b.p, b.p, 64, 48, 0, b.p, 1 << 20, None) == B.BPM_ERR_UNSUPPORTED_SIZE
    assert L.bpm_fft2(b.p, b.p, 64, 64, 2, b.p, 1 << 20, None) == B.BPM_ERR_INVALID_ARG
    assert L.bpm_pupil_spectrum(b.p, b.p, 64, 64, 0.2, 0.5, 1.33, float("nan"), b.p, None) == \
        B.BPM_ERR_NOT_FINITE
    assert L.bpm_pupil_phase_grad(None, b.p, 64, 64, b.p, None) == B.BPM_ERR_INVALID_ARG
    assert L.bpm_guide_star_phase(b.p, 64, 64, 0.2, 0.5, 1.36, 3.0, float("inf"), 0.0, b.p,
                                  None) == B.BPM_ERR_NOT_FINITE
    assert L.bpm_guide_star_phase(None, 64, 64, 0.2, 0.5, 1.36, 3.0, 0.0, 0.0, b.p,
                                  None) == B.BPM_ERR_INVALID_ARG
    assert L.bpm_guide_star_phase(b.p, 64, 96, 0.2, 0.5, 1.36, 3.0, 0.0, 0.0, b.p,
                                  None) == B.BPM_ERR_UNSUPPORTED_SIZE
    assert L.bpm_adam_step(b.p, b.p, b.p, b.p, 16, 0.1, 0, None) == B.BPM_ERR_INVALID_ARG
    assert L.bpm_adam_step(b.p, b.p, b.p, b.p, -1, 0.1, 1, None) == B.BPM_ERR_INVALID_ARG
    assert L.bpm_adam_step(b.p, b.p, b.p, b.p, 16, float("nan"), 1, None) == B.BPM_ERR_NOT_FINITE
    assert L.bpm_adam_step(b.p, None, b.p, b.p, 16, 0.1, 1, None) == B.BPM_ERR_INVALID_ARG
    assert L.bpm_adam_step(None, None, None, None, 0, 0.1, 1, None) == B.BPM_OK
    ws = L.bpm_pupil_fields_workspace_size(64, 64)
    assert ws > 0 and L.bpm_pupil_fields_workspace_size(64, 48) == 0
    assert L.bpm_pupil_fields(b.p, 64, 64, 0.2, 0.2, 0.5, 1.33, 0.6, 3, b.p, 2, 24, b.p, b.p, ws,
                              None) == B.BPM_ERR_INVALID_ARG
    assert L.bpm_pupil_fields(b.p, 64, 64, 0.2, 0.2, 0.5, 1.33, 0.6, 3, b.p, 2, 32, b.p, b.p,
                              ws - 1, None) == B.BPM_ERR_WORKSPACE
    assert L.bpm_zernike_workspace_size(32, 29) == 0 and L.bpm_zernike_workspace_size(32, 15) > 0
    zws = L.bpm_zernike_workspace_size(32, 15)
    # NA 0.05: the disc holds too few samples; NA 1.4 at dx 0.2: it leaves the window's band
    assert L.bpm_zernike_fit(b.p, 2, 32, 0.2, 0.5, 0.05, 15, b.p, None, b.p, zws,
                             None) == B.BPM_ERR_INVALID_ARG and b"samples" in L.bpm_last_error()
    assert L.bpm_zernike_fit(b.p, 2, 32, 0.2, 0.5, 1.4, 15, b.p, None, b.p, zws,
                             None) == B.BPM_ERR_INVALID_ARG and b"band" in L.bpm_last_error()
    assert L.bpm_zernike_fit(b.p, 2, 32, 0.2, 0.5, 0.6, 15, b.p, None, b.p, zws - 1,
                             None) == B.BPM_ERR_WORKSPACE
    assert L.bpm_camera_accumulate(b.p, None, b.p, 100, 64, 4, 32, b.p,
                                   None) == B.BPM_ERR_UNSUPPORTED_SIZE
    assert L.bpm_camera_accumulate(b.p, None, b.p, 128, 64, 64, 32, b.p,
                                   None) == B.BPM_ERR_INVALID_ARG      # one node row
    assert L.bpm_camera_accumulate(b.p, None, b.p, 128, 128, 32, 24, b.p,
                                   None) == B.BPM_ERR_INVALID_ARG
    assert L.bpm_camera_accumulate(b.p, b.p, b.p, 128, 128, 32, 32, b.p,
                                   None) == B.BPM_ERR_INVALID_ARG      # image aliases


def test_surrogate_validation(L):
    from paper_1706_02261_amd import _lib as B
    b = Buf(1 << 16)
    # sizes are pure host arithmetic
    assert L.psf_surrogate_param_count() > 0
    assert L.psf_surrogate_weights_bytes() % 256 == 0
    assert L.psf_surrogate_workspace_size(1, 1) > L.psf_surrogate_workspace_size(1, 0)
    assert L.psf_surrogate_workspace_size(-1, 0) == 0
    g = (ctypes.c_int * 15)()
    assert L.psf_surrogate_layer_geometry(0, g) == B.BPM_OK and list(g)[:6] == [1, 64, 32, 32, 8, 32]
    assert L.psf_surrogate_layer_geometry(6, g) == B.BPM_ERR_INVALID_ARG
    nbytes = L.psf_surrogate_weights_bytes()
    # wrong blob size, negative batch, missing workspace
    assert L.psf_surrogate_infer(b.p, nbytes - 1, b.p, b.p, 4, b.p, b.p, b.p, 1 << 20,
                                 None) == B.BPM_ERR_INVALID_ARG
    assert L.psf_surrogate_infer(b.p, nbytes, b.p, b.p, -1, b.p, b.p, b.p, 1 << 20,
                                 None) == B.BPM_ERR_INVALID_ARG
    assert L.psf_surrogate_infer(b.p, nbytes, b.p, b.p, 0, None, None, None, 0, None) == B.BPM_OK
    assert L.psf_surrogate_infer(b.p, nbytes, b.p, b.p, 4, b.p, b.p, b.p, 16,
                                 None) == B.BPM_ERR_WORKSPACE
    # training step: batch range, lr, step
    ws = L.psf_surrogate_workspace_size(8, 1)
    assert L.psf_surrogate_train_step(b.p, b.p, b.p, b.p, 0, 1e-3, 1.0, 1, b.p, None, b.p, ws,
                                      None) == B.BPM_ERR_INVALID_ARG
    assert L.psf_surrogate_train_step(b.p, b.p, b.p, b.p, 8, float("nan"), 1.0, 1, b.p, None,
                                      b.p, ws, None) == B.BPM_ERR_NOT_FINITE
    assert L.psf_surrogate_train_step(b.p, b.p, b.p, b.p, 8, 1e-3, 1.0, 0, b.p, None, b.p, ws,
                                      None) == B.BPM_ERR_INVALID_ARG
    # patch extraction: the 64-slice window must fit
    assert L.psf_extract_patches(b.p, 63, 32, 32, 0, b.p, 1, b.p, None) == B.BPM_ERR_INVALID_ARG
    assert L.psf_extract_patches(b.p, 70, 32, 32, 7, b.p, 1, b.p, None) == B.BPM_ERR_INVALID_ARG
    assert L.psf_extract_patches(b.p, 70, 32, 32, 6, b.p, 0, b.p, None) == B.BPM_OK


@pytest.mark.parametrize("geom,code", [
    ((1, 8, 8, 8, 6, 32, 3, 3, 3, 1, 1, 1, 1, 1, 1), "unsupported"),   # Ci not a multiple of 8
    ((1, 8, 8, 8, 8, 48, 3, 3, 3, 1, 1, 1, 1, 1, 1), "unsupported"),   # Co not 32 .. 256
    ((1, 8, 8, 8, 8, 32, 9, 3, 3, 1, 1, 1, 0, 1, 1), "invalid"),       # kernel larger than input
    ((1, 4, 4, 300, 8, 32, 1, 1, 1, 1, 1, 1, 0, 0, 0), "unsupported"),  # output rows over 128
    ((0, 8, 8, 8, 8, 32, 3, 3, 3, 1, 1, 1, 1, 1, 1), "invalid"),
])
def test_conv_geometry_validation(L, geom, code):
    from paper_1706_02261_amd import _lib as B
    b = Buf(1 << 16)
    g = (ctypes.c_int * 15)(*geom)
    want = B.BPM_ERR_UNSUPPORTED_SIZE if code == "unsupported" else B.BPM_ERR_INVALID_ARG
    assert L.psf_conv_forward(b.p, b.p, b.p, g, 0, b.p, None, None, b.p, 1 << 16, None) == want


def test_point_sources_validation(L):
    from paper_1706_02261_amd import _lib as B
    b = Buf()
    ws = L.bpm_point_sources_workspace_size(64, 64)
    assert ws > 0 and L.bpm_point_sources_workspace_size(48, 64) == 0
    assert L.bpm_point_sources(b.p, None, 4, 64, 64, 0.2, 0.5, 1.33, 0.0, 0.0, b.p, b.p, ws,
                               None) == B.BPM_ERR_NOT_FINITE
    assert L.bpm_point_sources(b.p, None, -1, 64, 64, 0.2, 0.5, 1.33, 0.6, 0.0, b.p, b.p, ws,
                               None) == B.BPM_ERR_INVALID_ARG
    assert L.bpm_point_sources(None, None, 4, 64, 64, 0.2, 0.5, 1.33, 0.6, 0.0, b.p, b.p, ws,
                               None) == B.BPM_ERR_INVALID_ARG
    assert L.bpm_point_sources(b.p, None, 4, 64, 64, 0.2, 0.5, 1.33, 0.6, 0.0, b.p, b.p, 8,
                               None) == B.BPM_ERR_WORKSPACE


def test_status_word_maps_to_device_error(L):
    """The sticky mask that the persistent kernels set when a wait gives up
    (word 0 of a workspace's status header) maps to BPM_ERR_DEVICE with a
    message naming the kind of wait; a clear mask is BPM_OK."""
    from paper_1706_02261_amd import _lib as B
    assert L.bpm_decode_status(0) == B.BPM_OK
    assert L.bpm_decode_status(1) == B.BPM_ERR_DEVICE
    assert b"grid-barrier" in L.bpm_last_error() and b"not valid" in L.bpm_last_error()
    assert L.bpm_decode_status(2) == B.BPM_ERR_DEVICE
    assert b"work-queue" in L.bpm_last_error()
    assert L.bpm_decode_status(3) == B.BPM_ERR_DEVICE
    msg = L.bpm_last_error()
    assert b"grid-barrier" in msg and b"work-queue" in msg
    assert L.bpm_decode_status(0x80) == B.BPM_ERR_DEVICE
    assert b"unknown" in L.bpm_last_error()


def test_workspace_status_validation(L):
    from paper_1706_02261_amd import _lib as B
    b = Buf()
    assert L.bpm_workspace_status(None, 4096, None) == B.BPM_ERR_WORKSPACE
    assert L.bpm_workspace_status(b.p, 255, None) == B.BPM_ERR_WORKSPACE
    assert L.bpm_workspace_status(b.p + 8, 4096, None) == B.BPM_ERR_WORKSPACE
    assert L.bpm_set_wait_limit(1 << 40) == B.BPM_ERR_INVALID_ARG
    assert L.bpm_set_wait_limit(0) == B.BPM_OK


def test_fallback_runs_keep_sources_apart():
    """Host grouping of the surrogate's fallback: every source in exactly one
    run, and two sources of one run more than the crop pitch apart along y or
    x, circularly (also across the wrap of the periodic field)."""
    import itertools
    from paper_1706_02261_amd.psfs import fallback_runs
    rng = np.random.default_rng(5)
    for n, m, sep in ((1024, 700, 32), (256, 200, 32), (64, 30, 32), (512, 300, 48)):
        yx = rng.integers(0, n, (m, 2))
        yx[:4] = [[0, 5], [n - 3, 5], [7, n - 1], [7, 2]]       # neighbours across the wrap
        runs = fallback_runs(yx, n, n, sep)
        assert sorted(np.concatenate(runs).tolist()) == list(range(m))
        for r in runs:
            for a, b in itertools.combinations(r, 2):
                d = np.abs(yx[a] - yx[b])
                d = np.minimum(d, n - d)
                assert d.max() > sep
    assert fallback_runs(np.zeros((0, 2), int), 64, 64) == []


def test_march_variant_choice_and_overrides(L):
    """Kernel choice of the forward march per shape: eligibility, the
    built-in choice and overrides (no device: the tiled two-field kernel,
    which needs the device's CU count, is never eligible here)."""
    from paper_1706_02261_amd import _lib as B
    assert L.bpm_march_variant_eligible(64, 64, 1, B.BPM_MARCH_ONE_PER_CU) == 1
    assert L.bpm_march_variant_eligible(256, 1024, 2, B.BPM_MARCH_TWO_PER_CU) == 0
    assert L.bpm_march_variant_eligible(512, 1024, 3, B.BPM_MARCH_TWO_PER_CU) == 1
    assert L.bpm_march_variant_eligible(512, 512, 9, B.BPM_MARCH_ONE_PER_CU) == 0
    assert L.bpm_march_variant_eligible(512, 512, 1, 7) == 0
    assert L.bpm_march_variant_eligible(1024, 128, 3, B.BPM_MARCH_SMALL_BLOCKS) == 1
    assert L.bpm_march_variant_eligible(2048, 512, 1, B.BPM_MARCH_SMALL_BLOCKS) == 0
    assert L.bpm_march_variant(100, 64, 1) == B.BPM_ERR_INVALID_ARG
    assert L.bpm_march_variant(512, 512, 1) == B.BPM_MARCH_SMALL_BLOCKS
    assert L.bpm_march_variant(1024, 1024, 1) == B.BPM_MARCH_ONE_PER_CU
    assert L.bpm_march_variant(512, 512, 2) == B.BPM_MARCH_TWO_PER_CU
    assert L.bpm_set_march_variant(512, 512, 2, B.BPM_MARCH_ONE_PER_CU) == B.BPM_OK
    assert L.bpm_march_variant(512, 512, 2) == B.BPM_MARCH_ONE_PER_CU
    assert L.bpm_march_variant(512, 512, 3) == B.BPM_MARCH_TWO_PER_CU     # other shape untouched
    assert L.bpm_set_march_variant(512, 512, 2, B.BPM_MARCH_AUTO) == B.BPM_OK
    assert L.bpm_march_variant(512, 512, 2) == B.BPM_MARCH_TWO_PER_CU
    assert L.bpm_set_march_variant(256, 256, 2, B.BPM_MARCH_TWO_PER_CU) == B.BPM_ERR_INVALID_ARG
    assert L.bpm_set_march_variant(256, 256, 2, 9) == B.BPM_ERR_INVALID_ARG
    assert L.bpm_set_march_variant(256, 256, 0, B.BPM_MARCH_AUTO) == B.BPM_ERR_INVALID_ARG


def test_adapted_march_validation(L):
    from paper_1706_02261_amd import _lib as B
    b = Buf()
    ws = L.bpm_workspace_size(64, 64, 2, 0)
    assert L.bpm_propagate_adapted(b.p, b.p, None, 64, 64, 2, 0.2, 0.2, 0.5, 1.33, b.p, None,
                                   b.p, ws, None) == B.BPM_ERR_INVALID_ARG
    assert L.bpm_propagate_adapted(b.p, b.p, b.p, 100, 64, 2, 0.2, 0.2, 0.5, 1.33, b.p, None,
                                   b.p, ws, None) == B.BPM_ERR_UNSUPPORTED_SIZE
    assert L.bpm_propagate_adapted(b.p, b.p, b.p, 64, 64, 2, 0.2, 0.2, 0.5, 1.33, b.p, None,
                                   b.p, 16, None) == B.BPM_ERR_WORKSPACE
    assert L.bpm_slice_means(b.p, 64, 64, -1, b.p, None) == B.BPM_ERR_INVALID_ARG
    assert L.bpm_slice_means(None, 64, 64, 3, b.p, None) == B.BPM_ERR_INVALID_ARG
    assert L.bpm_slice_means(b.p, 64, 48, 3, b.p, None) == B.BPM_ERR_UNSUPPORTED_SIZE
