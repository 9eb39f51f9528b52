"""GPU parity of the march with a locally adapted expansion of the refractive
index (bpm_propagate_adapted, bpm_slice_means) against the FP64 oracle.

The oracle receives the very dn_ref the GPU used (float32, upcast exactly).
Tolerances as the plain march's: the propagator is formed on the fly from an
FP64 kz and an FP32 phasor (relative error ~1e-7 per step), so short runs stay
within 2e-6 (field) / 4e-6 (intensity) and 64-step runs within 1e-4.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
LAM, N0 = 0.5, 1.33


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def case(nx, ny, steps, seed):
    rng = np.random.default_rng(seed)
    u0 = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
    dn = rng.uniform(0, 0.05, (steps, ny, nx)).astype(np.float32)
    ref = rng.uniform(-0.02, 0.06, steps).astype(np.float32)
    return u0, dn, ref


@pytest.mark.parametrize("nx,ny,steps,dx", [(64, 128, 5, 0.2), (256, 256, 7, 0.1),
                                            (512, 256, 4, 0.2), (1024, 1024, 3, 0.2),
                                            (2048, 64, 3, 0.2)])
def test_adapted_march_parity(nx, ny, steps, dx):
    import paper_1706_02261_amd as bpm
    u0, dn, ref = case(nx, ny, steps, seed=nx + 3 * ny + steps)
    out, inten, _ = bpm.propagate_adapted(torch.from_numpy(u0).cuda(), torch.from_numpy(dn).cuda(),
                                          dx, 0.2, LAM, N0, dn_ref=torch.from_numpy(ref).cuda())
    torch.cuda.synchronize()
    ru, ri = oracle.bpm_forward_adapted(u0, dn, ref, dx, 0.2, LAM, N0)
    eu, ei = rel(out.cpu().numpy(), ru), rel(inten.cpu().numpy(), ri)
    print(f"{nx} x {ny} x {steps}: field {eu:.2e} intensity {ei:.2e}")
    assert eu <= 2e-6 and ei <= 4e-6


def test_slice_means():
    import paper_1706_02261_amd as bpm
    rng = np.random.default_rng(2)
    dn = rng.uniform(-0.01, 0.05, (9, 512, 256)).astype(np.float32)
    m = bpm.slice_means(torch.from_numpy(dn).cuda()).cpu().numpy()
    ref = dn.astype(np.float64).mean(axis=(1, 2))
    assert np.abs(m - ref).max() <= 1e-7 * np.abs(ref).max() + 1e-12
    assert bpm.slice_means(torch.from_numpy(dn[:0]).cuda()).numel() == 0


def test_multiplexed_workload_with_slice_means():
    """The 512^2 multiplexed-PSF workload (first 64 slices), each slice
    expanded about its own mean index: <= 1e-4 against the oracle."""
    import paper_1706_02261_amd as bpm
    g, u0, dn = synth.config1(steps=64)
    out, inten, ref = bpm.propagate_adapted(torch.from_numpy(u0).cuda(),
                                            torch.from_numpy(dn).cuda(), g.dx, g.dz,
                                            g.wavelength, g.n0)
    torch.cuda.synchronize()
    ref_h = ref.cpu().numpy()
    assert np.abs(ref_h - dn.astype(np.float64).mean(axis=(1, 2))).max() <= 1e-8
    ru, ri = oracle.bpm_forward_adapted(u0, dn, ref_h, g.dx, g.dz, g.wavelength, g.n0)
    eu, ei = rel(out.cpu().numpy(), ru), rel(inten.cpu().numpy(), ri)
    print(f"512^2 x 64 slice means: field {eu:.2e} intensity {ei:.2e}")
    assert eu <= 1e-4 and ei <= 1e-4


def test_adapted_expansion_is_exact_in_a_homogeneous_slab():
    """A tilted plane wave through 32 slices of a medium at n0 + 0.05: the
    adapted march (reference = the slab's index) matches the exact phase
    dz N sqrt((n k0)^2 - kt^2); the plain march misses it by the known
    paraxial-screen error."""
    import paper_1706_02261_amd as bpm
    nx = ny = 256
    dx = dz = 0.2
    qx, qy = 60, 35
    y, x = np.mgrid[0:ny, 0:nx]
    u0 = np.exp(2j * np.pi * (qx * x / nx + qy * y / ny)).astype(np.complex64)
    c, steps = 0.05, 32
    dn = np.full((steps, ny, nx), c, np.float32)
    k0 = 2 * np.pi / LAM
    kt2 = (2 * np.pi * qx / (nx * dx)) ** 2 + (2 * np.pi * qy / (ny * dx)) ** 2
    exact = u0.astype(complex) * np.exp(1j * steps * dz * np.sqrt(((N0 + c) * k0) ** 2 - kt2))
    f, d = torch.from_numpy(u0).cuda(), torch.from_numpy(dn).cuda()
    ua, _, _ = bpm.propagate_adapted(f, d, dx, dz, LAM, N0, intensity=False)
    up, _ = bpm.propagate(f, d, dx, dz, LAM, N0, intensity=False)
    torch.cuda.synchronize()
    ea, ep = rel(ua.cpu().numpy(), exact), rel(up.cpu().numpy(), exact)
    print(f"homogeneous slab: adapted {ea:.2e}, plain {ep:.2e}")
    assert ea <= 2e-5 and ep >= 1e-2
