"""Pins of the adaptive-optics oracle (oracle/ao.py) and of the Perlin-noise
tissue generator.

* clear medium: the guide-star phase is the aiming tilt -(kx x_f + ky y_f)
  on every propagating mode, and the memory-effect persistence is exactly 1
  (a shifted entrance field gives the shifted focus), also in a medium that
  is invariant along the shift;
* scattering medium: the corrected focus intensity equals the Cauchy-Schwarz
  optimum (sum A |G|)^2 and exceeds that of random and aimed phases, and any
  small change of the phase lowers it;
* speckle autocorrelation: cosine fringes cos(a x) cos(b y) give
  C(d) = (cos(a d) + cos(b d)) / 2;
* mean free paths: one thin screen gives -ln |<exp(i k0 dz dn)>|^2;
* the memory effect on the Perlin tissue: the half-width of P(s) matches the
  speckle autocorrelation length within 25% (the paper's observation);
* Perlin noise: zero on lattice points, continuous, seeded; the phantom has
  mean n0 and standard deviation 0.03.
"""
import numpy as np

import synth
from oracle import ao

LAM, N0, DX, DZ = 0.5, 1.36, 0.2, 0.2


def small_case(n=64, steps=12, seed=0):
    g = synth.Geometry(n, n, steps, DX, DZ, LAM, N0)
    dn = synth.perlin_phantom(g, feature_um=2.0, gen=synth.rng(seed, 0)).astype(float)
    kx, ky, kz = ao.wavenumbers(n, n, DX, LAM, N0)
    kt2 = kx ** 2 + ky ** 2
    kmax = 2 * np.pi / LAM * 0.6
    amp = np.where(kt2 <= kmax ** 2, np.exp(-kt2 / kmax ** 2), 0.0)
    return g, dn, amp, steps * DZ


def test_clear_medium_guide_star_is_the_aiming_tilt():
    g, dn, amp, zf = small_case()
    focus = (21, 40)
    gs = ao.guide_star_gradient(np.zeros_like(dn), focus, DX, DZ, LAM, N0)
    phi = ao.guide_star_phase(gs, DX, LAM, N0, zf)
    aim = ao.aim_phase(g.nx, g.ny, DX, LAM, N0, focus)
    _, _, kz = ao.wavenumbers(g.nx, g.ny, DX, LAM, N0)
    prop = kz > 0
    assert np.abs(ao.wrap(phi - aim)[prop]).max() <= 1e-9
    # and the aimed clear-medium field focuses on that pixel
    inten = np.abs(ao.exit_field(amp, aim, np.zeros_like(dn), DX, DZ, LAM, N0, zf)) ** 2
    assert np.unravel_index(np.argmax(inten), inten.shape) == focus


def test_correction_reaches_the_cauchy_schwarz_optimum():
    g, dn, amp, zf = small_case(seed=1)
    focus = (g.ny // 2, g.nx // 2)
    gs = ao.guide_star_gradient(dn, focus, DX, DZ, LAM, N0)
    best = ao.optimum_intensity(amp, gs)

    def focus_intensity(phi):
        u = ao.exit_field(amp, phi, dn, DX, DZ, LAM, N0, zf)
        return abs(u[focus]) ** 2

    phi_star = ao.guide_star_phase(gs, DX, LAM, N0, zf)
    assert abs(focus_intensity(phi_star) / best - 1) <= 1e-10
    rng = np.random.default_rng(2)
    assert focus_intensity(ao.aim_phase(g.nx, g.ny, DX, LAM, N0, focus)) < best
    for _ in range(5):
        assert focus_intensity(rng.uniform(-np.pi, np.pi, amp.shape)) < best
        assert focus_intensity(phi_star + 0.05 * rng.standard_normal(amp.shape)) < best


def test_memory_effect_is_exact_in_clear_and_shift_invariant_media():
    g, dn, amp, zf = small_case(seed=3)
    focus = (20, 30)
    shifts = [(0, 1), (0, 5), (3, 0), (-4, 7)]
    gs = ao.guide_star_gradient(np.zeros_like(dn), focus, DX, DZ, LAM, N0)
    P, _ = ao.memory_effect(amp, gs, np.zeros_like(dn), focus, shifts, DX, DZ, LAM, N0, zf)
    assert np.abs(P - 1).max() <= 1e-10
    # a medium that varies along y only is invariant under x shifts
    layered = np.repeat(dn[:, :, :1], g.nx, axis=2)
    gs = ao.guide_star_gradient(layered, focus, DX, DZ, LAM, N0)
    P, _ = ao.memory_effect(amp, gs, layered, focus, [(0, s) for s in (1, 3, 9, 17)], DX, DZ,
                            LAM, N0, zf)
    assert np.abs(P - 1).max() <= 1e-10
    P, _ = ao.memory_effect(amp, gs, layered, focus, [(5, 0)], DX, DZ, LAM, N0, zf)
    assert abs(P[0] - 1) > 0.05          # no invariance along y


def test_speckle_autocorrelation_of_cosine_fringes():
    n = 64
    y, x = np.mgrid[0:n, 0:n]
    a, b = 2 * np.pi * 4 / n, 2 * np.pi * 6 / n
    inten = 2.0 + np.cos(a * x) * np.cos(b * y)
    C = ao.speckle_autocorrelation(inten, 10)
    d = np.arange(11)
    assert np.abs(C - 0.5 * (np.cos(a * d) + np.cos(b * d))).max() <= 1e-12


def test_mean_free_paths_of_one_thin_screen():
    rng = np.random.default_rng(4)
    dn = rng.normal(0, 0.05, (1, 64, 64))
    pw = ao.plane_wave_speckle(dn, DX, DZ, LAM, N0)
    k0 = 2 * np.pi / LAM
    ref = -np.log(abs(np.mean(np.exp(1j * k0 * DZ * dn[0]))) ** 2)
    assert abs(ao.mean_free_paths(pw) - ref) <= 1e-10
    assert abs(ao.mean_free_paths(ao.plane_wave_speckle(np.full((3, 32, 32), 0.02), DX, DZ, LAM,
                                                        N0))) <= 1e-12


def half_width(c):
    for i in range(1, len(c)):
        if c[i] < 0.5:
            return i - 1 + (c[i - 1] - 0.5) / (c[i - 1] - c[i])
    return float("inf")


def test_memory_effect_range_is_the_speckle_correlation_length():
    """128^2 x 80 Perlin tissue (about five mean free paths): persistence of the
    shifted focus against the plane-wave speckle autocorrelation."""
    g, dn, amp, zf = synth.ao_workload(128, 80)
    dn = dn.astype(float)
    f = (g.ny // 2, g.nx // 2)
    gs = ao.guide_star_gradient(dn, f, g.dx, g.dz, g.wavelength, g.n0)
    shifts = [(0, s) for s in range(1, 7)] + [(s, 0) for s in range(1, 7)]
    P, _ = ao.memory_effect(amp, gs, dn, f, shifts, g.dx, g.dz, g.wavelength, g.n0, zf)
    Pm = np.r_[1.0, 0.5 * (P[:6] + P[6:])]
    pw = ao.plane_wave_speckle(dn, g.dx, g.dz, g.wavelength, g.n0)
    C = ao.speckle_autocorrelation(np.abs(pw) ** 2, 6)
    mfp = ao.mean_free_paths(pw)
    print(f"mfp {mfp:.2f} half-widths P {half_width(Pm):.2f} C {half_width(C):.2f} px")
    assert mfp > 3.0
    assert abs(half_width(Pm) / half_width(C) - 1) <= 0.25


def test_perlin_noise_lattice_zeros_continuity_and_seed():
    p = synth.perlin_noise((9, 40, 40), 4.0, np.random.default_rng(0))
    assert np.abs(p[::4, ::4, ::4]).max() <= 1e-12          # gradient noise vanishes on the lattice
    assert 0.2 <= np.abs(p).max() <= 1.0
    # the quintic fade makes the noise C2 across cell faces: on a 16-voxel
    # lattice the second differences stay O(1 / 16^2) (a linear blend would
    # jump by O(1 / 16) at every face)
    s = synth.perlin_noise((3, 64, 64), 16.0, np.random.default_rng(0))
    assert np.abs(np.diff(s, n=2, axis=2)).max() <= 0.05
    assert np.abs(np.diff(s, n=2, axis=1)).max() <= 0.05
    q = synth.perlin_noise((9, 40, 40), 4.0, np.random.default_rng(0))
    assert np.array_equal(p, q)
    r = synth.perlin_noise((9, 40, 40), 4.0, np.random.default_rng(1))
    assert not np.array_equal(p, r)


def test_perlin_phantom_statistics():
    g = synth.Geometry(64, 64, 16, DX, DZ, LAM, N0)
    dn = synth.perlin_phantom(g)
    assert dn.dtype == np.float32 and dn.shape == (16, 64, 64)
    assert abs(float(dn.mean())) <= 1e-6 and abs(float(dn.std()) - 0.03) <= 1e-6
