"""The allocation-free forward march (bpm_propagate_noalloc) through the C
ABI: two calls in a row on the library's per-GPU plan memory, the second with
a smaller field, each bit for bit equal to bpm_propagate with a workspace;
a field above the limit is rejected before any launch."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def case(nx, ny, steps, seed):
    rng = np.random.default_rng(seed)
    u0 = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
    dn = rng.uniform(0, 0.05, (steps, ny, nx)).astype(np.float32)
    return torch.from_numpy(u0).cuda(), torch.from_numpy(dn).cuda()


def noalloc(L, f, d, out, inten, dx=0.2):
    ny, nx = f.shape
    return L.bpm_propagate_noalloc(f.data_ptr(), d.data_ptr(), nx, ny, d.shape[0], dx, 0.2, 0.5,
                                   1.33, out.data_ptr(), None if inten is None else inten.data_ptr(),
                                   None)


def test_noalloc_march_equals_the_workspace_march():
    import paper_1706_02261_amd as bpm
    from paper_1706_02261_amd import _lib
    L = _lib.lib()
    assert L.bpm_noalloc_scratch_bytes() >= bpm.workspace_size(1024, 1024, 1)
    for k, (nx, ny, steps, dx) in enumerate([(1024, 1024, 4, 0.2), (256, 128, 7, 0.1)]):
        print(f"call {k}: {nx} x {ny} x {steps}", flush=True)
        f, d = case(nx, ny, steps, seed=k + 3)
        out = torch.full_like(f, 7.0)
        inten = torch.full((steps, ny, nx), 7.0, device="cuda")
        assert noalloc(L, f, d, out, inten, dx) == 0, L.bpm_last_error()
        torch.cuda.synchronize()
        ref, ref_i = bpm.propagate(f, d, dx, 0.2, 0.5, 1.33)
        torch.cuda.synchronize()
        assert torch.equal(out, ref) and torch.equal(inten, ref_i)
    # without the intensity volume, in place
    f, d = case(512, 512, 3, seed=9)
    ref, _ = bpm.propagate(f, d, 0.2, 0.2, 0.5, 1.33, intensity=False)
    assert noalloc(L, f, d, f, None) == 0
    torch.cuda.synchronize()
    assert torch.equal(f, ref)


def test_noalloc_rejects_fields_above_its_limit():
    from paper_1706_02261_amd import _lib
    L = _lib.lib()
    f, d = case(2048, 1024, 1, seed=1)
    out = torch.full_like(f, 7.0)
    rc = noalloc(L, f, d, out, None)
    assert rc == _lib.BPM_ERR_UNSUPPORTED_SIZE and b"1024 x 1024" in L.bpm_last_error()
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
