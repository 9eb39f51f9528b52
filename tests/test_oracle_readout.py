"""Pins of the oracle's PSF readout (refocusing lens of the detection path).

* free space: after a dn = 0 march the back-propagated in-focus plane is the
  source field itself (H^L conj(H)^L = 1 on propagating modes);
* free-space propagation keeps the energy of every refocused plane;
* an aberration-free pupil gives I(x, -z) = I(-x, z) about the source;
* modes outside the detection NA are cut.
"""
import numpy as np

import oracle
import synth

LAM, N0, NA = 0.5, 1.33, 0.6


def sources_grid(n, pitch):
    c = np.arange(pitch // 2, n, pitch)
    yy, xx = np.meshgrid(c, c, indexing="ij")
    return np.stack([yy.ravel(), xx.ravel()], 1)


def test_in_focus_plane_is_the_source_field():
    n, L, dz = 64, 9, 0.2
    src = sources_grid(n, 32)
    one = np.fft.ifft2(synth.point_source_spectrum(n, n, 0.2, LAM, N0, NA, 0.0))  # float64
    u0 = sum(np.exp(1j * ph) * np.roll(one, tuple(p), axis=(0, 1))
             for p, ph in zip(src, [0.3, 1.1, 2.0, 2.9]))
    exit_, _ = oracle.bpm_forward(u0, np.zeros((L, n, n)), 0.2, dz, LAM, N0, intensity=False)
    psf = oracle.psf_readout(exit_, 0.2, dz, LAM, N0, NA, L, src, planes=8, crop=32)
    for s, (sy, sx) in enumerate(src):
        ys = (np.arange(32) + sy - 16) % n
        xs = (np.arange(32) + sx - 16) % n
        ref = np.abs(u0[np.ix_(ys, xs)]) ** 2
        assert np.abs(psf[s, 4] - ref).max() <= 1e-12 * ref.max()


def test_energy_of_every_plane_is_conserved():
    n = 64
    src = sources_grid(n, 32)
    rng = np.random.default_rng(1)
    dn = rng.uniform(0, 0.05, (7, n, n))
    u0 = synth.multiplexed_field(n, n, 0.2, LAM, N0, NA, 0.0, src, rng.uniform(0, 6, len(src)))
    exit_, _ = oracle.bpm_forward(u0, dn, 0.2, 0.2, LAM, N0, intensity=False)
    psf = oracle.psf_readout(exit_, 0.2, 0.2, LAM, N0, NA, 7, src, planes=16, crop=32)
    energy = psf.sum(axis=(0, 2, 3))          # crops tile the plane
    assert np.abs(energy / energy[0] - 1).max() <= 1e-12


def test_defocus_mirror_symmetry():
    n = 64
    src = np.array([[32, 32]])
    u0 = synth.point_source_field(n, n, 0.2, LAM, N0, NA, 0.0, centre=(32, 32)).astype(complex)
    exit_, _ = oracle.bpm_forward(u0, np.zeros((5, n, n)), 0.2, 0.2, LAM, N0, intensity=False)
    psf = oracle.psf_readout(exit_, 0.2, 0.2, LAM, N0, NA, 5, src, planes=32, crop=32)[0]
    for m in range(1, 16):
        a = psf[16 + m, 1:, 1:]
        b = psf[16 - m, 1:, 1:][::-1, ::-1]
        assert np.abs(a - b).max() <= 1e-12 * psf.max()


def test_modes_outside_the_na_are_cut():
    n = 64
    y, x = np.mgrid[0:n, 0:n]
    inside = np.exp(2j * np.pi * (3 * x / n))            # 3 / 12.8 um^-1 < NA / lambda
    outside = np.exp(2j * np.pi * (20 * x / n))          # 20 / 12.8 um^-1 > NA / lambda
    psf_in = oracle.psf_readout(inside, 0.2, 0.2, LAM, N0, NA, 0, [[0, 0]], planes=2, crop=8)
    psf_out = oracle.psf_readout(outside, 0.2, 0.2, LAM, N0, NA, 0, [[0, 0]], planes=2, crop=8)
    assert np.abs(psf_in - 1).max() <= 1e-12
    assert np.abs(psf_out).max() <= 1e-24


def test_refocus_planes_lie_downstream_of_the_source():
    """Plane m of the readout is the field m dz past the source plane.

    The source is a converging spectrum A(k) exp(-i kz q dz), written out
    here: it focuses q dz downstream of its plane under the march's
    propagator (whose sign the single-mode phase pin fixes).  Read out with
    no back-propagation, its on-axis peak must sit at plane planes/2 + q, and
    every plane m >= 1 must equal the free-space march of the source through
    m slices; a readout that refocused upstream (the sign of m flipped) puts
    the peak at planes/2 - q and fails both."""
    n, dz, planes = 64, 0.2, 32
    k0 = 2 * np.pi / LAM
    f = np.fft.fftfreq(n, d=0.2) * 2 * np.pi
    kx, ky = np.meshgrid(f, f)
    kt2 = kx ** 2 + ky ** 2
    kmax = k0 * NA
    kz = np.sqrt(np.maximum((N0 * k0) ** 2 - kt2, 0.0))
    amp = np.where(kt2 <= kmax ** 2, np.exp(-kt2 / kmax ** 2), 0.0)
    for q in (5, -7):
        u0 = np.fft.ifft2(amp * np.exp(-1j * kz * q * dz))
        u0 = np.roll(u0, (n // 2, n // 2), axis=(0, 1))      # source at the grid centre
        psf = oracle.psf_readout(u0, 0.2, dz, LAM, N0, NA, 0, [[n // 2, n // 2]],
                                 planes=planes, crop=32)[0]
        axis = psf[:, 16, 16]
        assert int(np.argmax(axis)) == planes // 2 + q
        steps = planes // 2 - 1
        _, inten = oracle.bpm_forward(u0, np.zeros((steps, n, n)), 0.2, dz, LAM, N0)
        for m in range(1, steps + 1):
            ref = inten[m - 1][n // 2 - 16:n // 2 + 16, n // 2 - 16:n // 2 + 16]
            assert np.abs(psf[planes // 2 + m] - ref).max() <= 1e-12 * ref.max()
