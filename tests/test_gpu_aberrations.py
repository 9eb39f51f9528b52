"""GPU parity of the aberration maps (bpm_pupil_fields, bpm_zernike_fit) with
the FP64 oracle.

* pupil fields of a random exit field (windows that wrap around the grid
  edge, crops 16 / 32 / 64, with and without back-propagation);
* the Zernike fit of the same complex64 pupil fields on both sides, on the
  aberrated pupils of a sphere phantom and on synthetic pupils with wrapped
  tilts;
* a whole aberration map (sources on a grid, one multiplexed march) of a
  sphere phantom against the oracle chain, and the tilt map of a
  clear-medium run with displaced sources.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import zernike as zo

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
LAM, N0, NA, DX, DZ = 0.5, 1.33, 0.6, 0.2, 0.2


def to_gpu(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype)).cuda()


def cpu(t):
    return t.cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def optics():
    from paper_1706_02261_amd import psfs
    return psfs.Optics(DX, DZ, LAM, N0, NA)


@pytest.mark.parametrize("nx,ny,crop,back", [(256, 128, 32, 7), (128, 128, 16, 0),
                                             (256, 256, 64, 12), (64, 512, 32, 3)])
def test_pupil_fields(nx, ny, crop, back):
    from paper_1706_02261_amd import aberrations
    rng = np.random.default_rng(nx + ny + crop)
    u = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
    src = np.array([[ny // 2, nx // 2], [3, 5], [ny - 2, nx - 9], [ny // 3, 0]], np.int32)
    got = cpu(aberrations.pupil_fields(to_gpu(u, np.complex64), to_gpu(src, np.int32), back,
                                       optics(), crop))
    ref = zo.pupil_fields(u, DX, DZ, LAM, N0, NA, back, src, crop)
    assert got.shape == (4, crop, crop)
    assert rel(got, ref) <= 2e-5


def sphere_pupils(n=256, steps=80, pitch=64, seed=2):
    g = synth.Geometry(n, n, steps, DX, DZ, LAM, N0)
    dn = synth.sphere_phantom(g, 80, (1.0, 4.0), (0.01, 0.05), synth.rng(seed, 0))
    c = np.arange(pitch // 2, n, pitch)
    src = np.stack(np.meshgrid(c, c, indexing="ij"), -1).reshape(-1, 2).astype(np.int32)
    u0 = oracle.point_sources(n, n, DX, LAM, N0, NA, 0.0, src)
    exit_, _ = oracle.bpm_forward(u0, dn.astype(float), DX, DZ, LAM, N0, intensity=False)
    return dn, src, exit_


def test_zernike_fit_same_pupils():
    """Both sides fit the same complex64 pupil fields."""
    from paper_1706_02261_amd import aberrations
    _, src, exit_ = sphere_pupils()
    X = zo.pupil_fields(exit_, DX, DZ, LAM, N0, NA, 80, src, 32).astype(np.complex64)
    # and synthetic pupils whose tilt wraps several times across the disc
    mask, rho, theta = zo.disc(32, DX, LAM, NA)
    sign = (-1.0) ** (np.arange(32)[:, None] + np.arange(32)[None, :])
    K0 = 2 * np.pi / LAM
    extra = [np.where(mask, np.exp(1j * (-K0 * NA * rho * (np.cos(theta) * sx + np.sin(theta) * sy)
                                         + 0.4 * rho ** 2 * np.cos(2 * theta))), 0) * sign
             for sx, sy in [(0.9, -0.3), (-0.6, 0.7)]]
    X = np.concatenate([X, np.array(extra, np.complex64)])
    c, rms = aberrations.zernike_fit(to_gpu(X, np.complex64), optics(), 21)
    c_o, rms_o = zo.zernike_fit(X.astype(complex), DX, LAM, NA, 21)
    err = np.abs(cpu(c) - c_o).max()
    print(f"max |dc| {err:.2e} rad, rms {cpu(rms)[:4]} vs {rms_o[:4]}")
    assert err <= 2e-5 and np.abs(cpu(rms) - rms_o).max() <= 2e-5


def test_zernike_map_of_a_sphere_phantom():
    from paper_1706_02261_amd import aberrations
    dn, src, exit_ = sphere_pupils()
    maps, rms, src_g = aberrations.zernike_map(to_gpu(dn, np.float32), 0, pitch=64,
                                               optics=optics(), n_modes=15, crop=32)
    assert np.array_equal(cpu(src_g), src)
    X = zo.pupil_fields(exit_, DX, DZ, LAM, N0, NA, 80, src, 32)
    c_o, rms_o = zo.zernike_fit(X, DX, LAM, NA, 15)
    got = cpu(maps).reshape(15, -1).T
    err = np.abs(got - c_o).max()
    print(f"map: max |dc| {err:.2e} rad over {len(src)} sources; |c| up to {np.abs(c_o).max():.2f}")
    assert err <= 2e-4 and np.abs(cpu(rms).ravel() - rms_o).max() <= 2e-4
    assert np.abs(c_o[:, 1:]).max() > 0.05        # the phantom does aberrate


def test_clear_medium_tilt_map():
    """Sources displaced by s pixels from the window centres: c_2 = -k0 NA s dx / 2."""
    from paper_1706_02261_amd import aberrations
    from paper_1706_02261_amd import bpm
    n, steps = 256, 12
    c = np.arange(32, n, 64)
    src = np.stack(np.meshgrid(c, c, indexing="ij"), -1).reshape(-1, 2).astype(np.int32)
    shift = np.tile([0, 1, -1, 2], 4)
    placed = (src + np.stack([np.zeros(16, int), shift], 1)).astype(np.int32)
    u0 = bpm.point_sources(to_gpu(placed, np.int32), n, n, DX, LAM, N0, NA, 0.0)
    exit_, _ = bpm.propagate(u0, torch.zeros((steps, n, n), dtype=torch.float32, device="cuda"),
                             DX, DZ, LAM, N0, intensity=False)
    X = aberrations.pupil_fields(exit_, to_gpu(src, np.int32), steps, optics(), 32)
    cf, rms = aberrations.zernike_fit(X, optics(), 10)
    cf = cpu(cf)
    ref = -2 * np.pi / LAM * NA * shift * DX / 2
    assert np.abs(cf[:, 1] - ref).max() <= 0.01 + 0.01 * np.abs(ref).max()
    assert np.abs(cf[:, 2:]).max() <= 2e-2 and cpu(rms).max() <= 0.03


def test_empty_source_lists():
    from paper_1706_02261_amd import aberrations
    u = torch.zeros((64, 64), dtype=torch.complex64, device="cuda")
    X = aberrations.pupil_fields(u, torch.zeros((0, 2), dtype=torch.int32, device="cuda"), 3,
                                 optics(), 32)
    assert X.shape == (0, 32, 32)
    c, rms = aberrations.zernike_fit(X, optics(), 10)
    assert c.shape == (0, 10) and rms.shape == (0,)
