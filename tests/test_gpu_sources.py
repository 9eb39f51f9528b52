"""GPU parity of the multiplexed point-source builder and of the surrogate's
patch extraction (bit-exact gather) with the oracle and plain indexing."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
LAM, N0, NA = 0.5, 1.33, 0.6


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("nx,ny,n_src,z_d", [(128, 128, 16, 0.0), (256, 64, 7, 2.0),
                                            (64, 64, 1, -1.0), (1024, 1024, 1024, 0.0)])
def test_point_sources(nx, ny, n_src, z_d):
    import paper_1706_02261_amd as bpm
    gen = np.random.default_rng(nx + n_src)
    pos = np.stack([gen.integers(0, ny, n_src), gen.integers(0, nx, n_src)], 1).astype(np.int32)
    ph = gen.uniform(0, 2 * np.pi, n_src).astype(np.float32)
    u = bpm.point_sources(torch.from_numpy(pos).cuda(), nx, ny, 0.2, LAM, N0, NA, z_d,
                          phases=torch.from_numpy(ph).cuda())
    torch.cuda.synchronize()
    u = u.cpu().numpy()
    if nx * ny * n_src <= 1 << 22:
        ref = oracle.point_sources(nx, ny, 0.2, LAM, N0, NA, z_d, pos, ph.astype(np.float64))
    else:  # the direct shifted sum is slow at this size: the generator's comb convolution
        ref = synth.multiplexed_field(nx, ny, 0.2, LAM, N0, NA, z_d, pos, ph.astype(np.float64))
    assert rel(u, ref) <= 1e-5


def test_point_sources_empty_and_coinciding():
    import paper_1706_02261_amd as bpm
    z = bpm.point_sources(torch.zeros((0, 2), dtype=torch.int32, device="cuda"), 64, 64, 0.2,
                          LAM, N0, NA, 0.0)
    pos = torch.tensor([[10, 20], [10, 20], [74, 84]], dtype=torch.int32, device="cuda")
    u = bpm.point_sources(pos, 64, 64, 0.2, LAM, N0, NA, 0.0)
    torch.cuda.synchronize()
    assert float(z.abs().max()) == 0.0
    ref = 3 * oracle.point_sources(64, 64, 0.2, LAM, N0, NA, 0.0, [(10, 20)])
    assert rel(u.cpu().numpy(), ref) <= 1e-5


def test_extract_patches_bit_exact():
    from paper_1706_02261_amd import surrogate as S
    gen = np.random.default_rng(3)
    nz, ny, nx = 70, 96, 128
    dn = gen.standard_normal((nz, ny, nx)).astype(np.float32)
    src = np.array([[0, 0], [95, 127], [50, 64], [5, 120], [-3, 130]], dtype=np.int32)
    for z0 in (0, 6):
        got = S.extract_patches(torch.from_numpy(dn).cuda(), torch.from_numpy(src).cuda(), z0)
        torch.cuda.synchronize()
        yy = (src[:, 0, None] - 16 + np.arange(32)[None]) % ny
        xx = (src[:, 1, None] - 16 + np.arange(32)[None]) % nx
        ref = np.stack([dn[z0:z0 + 64][:, yy[s][:, None], xx[s][None, :]] for s in range(len(src))])
        assert np.array_equal(got.cpu().numpy(), ref)
