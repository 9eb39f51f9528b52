"""Pins of the oracle's forward march against closed forms and invariants.

None of these re-type the oracle's loop: each compares it with something the
physics or the mathematics fixes independently (plane-wave dispersion,
Jacobi-Anger expansion, paraxial Gaussian-beam width, exact lattice counts,
explicit DFT matrices, linearity, Parseval).
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy import special

import oracle
import synth

TWO_PI = 2 * np.pi


def kz_of(m, l, nx, ny, dx, lam, n0):
    """Plane-wave dispersion relation kz = sqrt((n0 k0)^2 - kx^2 - ky^2)."""
    k = n0 * TWO_PI / lam
    kx = TWO_PI * m / (nx * dx)
    ky = TWO_PI * l / (ny * dx)
    return np.sqrt(k * k - kx * kx - ky * ky + 0j)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ---------------------------------------------------------------------------
# homogeneous medium (the propagator and screen constants)

def test_homogeneous_plane_wave_phase():
    """u0 = 1 in a medium of index n0 + c: after N steps u = exp(i k0 (n0+c) N dz)."""
    nx, ny, steps, dx, dz, lam, n0, c = 32, 16, 7, 0.2, 0.3, 0.5, 1.33, 0.021
    u0 = np.ones((ny, nx), complex)
    dn = np.full((steps, ny, nx), c)
    u, inten = oracle.bpm_forward(u0, dn, dx, dz, lam, n0)
    expect = np.exp(1j * TWO_PI / lam * (n0 + c) * steps * dz)
    assert np.abs(u - expect).max() <= 1e-13
    assert np.abs(inten - 1).max() <= 1e-13


@pytest.mark.parametrize("m,l", [(3, -2), (-7, 5), (15, 0), (0, -8)])
def test_single_mode_phase(m, l):
    """A single DFT mode q advances by exp(i dz (kz(q) + k0 c)) per step."""
    nx, ny, steps, dx, dz, lam, n0, c = 32, 16, 5, 0.2, 0.2, 0.5, 1.33, 0.013
    y, x = np.mgrid[0:ny, 0:nx]
    u0 = np.exp(TWO_PI * 1j * (m * x / nx + l * y / ny))
    dn = np.full((steps, ny, nx), c)
    u, _ = oracle.bpm_forward(u0, dn, dx, dz, lam, n0)
    kz = kz_of(m, l, nx, ny, dx, lam, n0)
    expect = np.exp(1j * steps * dz * (kz + TWO_PI / lam * c)) * u0
    assert np.abs(u - expect).max() <= 1e-12


def test_evanescent_mode_is_cut():
    """A mode with kx^2 + ky^2 > k^2 is removed by the first step."""
    nx, ny, dx, dz, lam, n0 = 64, 64, 0.1, 0.1, 0.5, 1.33  # cut-off radius 17.0 px
    y, x = np.mgrid[0:ny, 0:nx]
    u0 = np.exp(TWO_PI * 1j * (20 * x / nx + 3 * y / ny))
    u, _ = oracle.bpm_forward(u0, np.zeros((1, ny, nx)), dx, dz, lam, n0)
    assert np.abs(u).max() <= 1e-13
    u0 = np.exp(TWO_PI * 1j * (16 * x / nx + 3 * y / ny))  # 16.3 px: propagates
    u, _ = oracle.bpm_forward(u0, np.zeros((1, ny, nx)), dx, dz, lam, n0)
    assert np.abs(np.abs(u) - 1).max() <= 1e-13


@pytest.mark.parametrize("n,dx,frac", [(128, Fraction("0.1"), 0.222), (512, Fraction("0.2"), 0.858),
                                       (1024, Fraction("0.2"), 0.858)])
def test_propagating_mode_count_exact(n, dx, frac):
    """Number of propagating modes = lattice points in the disc
    (m/N)^2 + (l/N)^2 <= (n0 dx / lambda)^2, counted in exact rationals."""
    n0, lam = Fraction("1.33"), Fraction("0.5")
    r2 = (n0 * dx / lam) ** 2 * n * n       # radius^2 in lattice units
    count = 0
    for l in range(-n // 2, n // 2):
        rem = r2 - l * l
        if rem < 0:
            continue
        # number of integers m in [-n/2, n/2) with m^2 <= rem
        mm = int(np.floor(np.sqrt(float(rem))))
        while (mm + 1) ** 2 <= rem:
            mm += 1
        while mm * mm > rem:
            mm -= 1
        lo, hi = max(-mm, -n // 2), min(mm, n // 2 - 1)
        count += max(0, hi - lo + 1)
    h = oracle.propagator(n, n, float(dx), 0.2, float(lam), float(n0))
    assert int((np.abs(h) > 0).sum()) == count
    assert abs(count / n ** 2 - frac) < 2e-3
    assert np.abs(np.abs(h[np.abs(h) > 0]) - 1).max() <= 1e-15


def test_composition_in_free_space():
    """dn = 0: N steps of dz equal one step of N dz (exact exponential law)."""
    nx, ny, steps = 64, 32, 9
    rng = np.random.default_rng(3)
    u0 = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    a, _ = oracle.bpm_forward(u0, np.zeros((steps, ny, nx)), 0.15, 0.2, 0.5, 1.33)
    b, _ = oracle.bpm_forward(u0, np.zeros((1, ny, nx)), 0.15, 0.2 * steps, 0.5, 1.33)
    assert rel(a, b) <= 1e-12


# ---------------------------------------------------------------------------
# energy

def test_parseval_all_modes_propagate():
    """dx >= lambda / (sqrt 2 n0): every mode propagates, the step is unitary."""
    nx, ny, steps = 64, 32, 20
    rng = np.random.default_rng(4)
    u0 = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    dn = rng.uniform(0, 0.05, (steps, ny, nx))
    u, inten = oracle.bpm_forward(u0, dn, 0.3, 0.2, 0.5, 1.33)
    e0 = np.sum(np.abs(u0) ** 2)
    assert abs(np.sum(np.abs(u) ** 2) / e0 - 1) <= 1e-13
    assert np.abs(inten.sum(axis=(1, 2)) / e0 - 1).max() <= 1e-13


def test_parseval_with_evanescent_cut():
    """One step keeps (1/N) sum over propagating modes of |DFT u0|^2."""
    nx = ny = 64
    dx, lam, n0 = Fraction("0.1"), Fraction("0.5"), Fraction("1.33")
    rng = np.random.default_rng(5)
    u0 = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    dn = rng.uniform(0, 0.05, (1, ny, nx))
    u, _ = oracle.bpm_forward(u0, dn, float(dx), 0.1, float(lam), float(n0))
    r2 = (n0 * dx / lam) ** 2
    m = np.fft.fftfreq(nx) * nx
    mask = np.array([[Fraction(int(a), nx) ** 2 + Fraction(int(b), ny) ** 2 <= r2 for a in m]
                     for b in m])
    spec = np.fft.fft2(u0)
    expect = np.sum(np.abs(spec[mask]) ** 2) / (nx * ny)
    assert abs(np.sum(np.abs(u) ** 2) / expect - 1) <= 1e-13


# ---------------------------------------------------------------------------
# screen-propagation coupling

def test_thin_grating_jacobi_anger():
    """u0 = 1, dn[0] = A cos(2 pi p x / Nx), dn[j>0] = 0.  After the first
    screen the field is exp(i k dz) sum_m i^m J_m(k0 dz A) exp(i m p theta);
    the remaining N-1 steps advance order m by exp(i dz kz(m p))."""
    nx, ny, steps, dx, dz, lam, n0, amp, p = 64, 8, 6, 0.2, 0.2, 0.5, 1.33, 0.05, 3
    x = np.arange(nx)
    dn = np.zeros((steps, ny, nx))
    dn[0] = amp * np.cos(TWO_PI * p * x / nx)[None, :]
    u, _ = oracle.bpm_forward(np.ones((ny, nx), complex), dn, dx, dz, lam, n0)
    k0 = TWO_PI / lam
    phi0 = k0 * dz * amp
    kz0 = kz_of(0, 0, nx, ny, dx, lam, n0)
    row = np.zeros(nx, complex)
    for m in range(-10, 11):           # |m p| <= 30 < Nx/2: no aliasing
        row += (1j ** m * special.jv(m, phi0) * np.exp(1j * (steps - 1) * dz *
                kz_of(m * p, 0, nx, ny, dx, lam, n0)) * np.exp(TWO_PI * 1j * m * p * x / nx))
    expect = np.exp(1j * dz * kz0) * np.broadcast_to(row, (ny, nx))
    assert np.abs(u - expect).max() <= 1e-12


# ---------------------------------------------------------------------------
# physical units: paraxial Gaussian beam

def test_gaussian_beam_width():
    """A waist w0 = 2 um in n0 = 1.33 spreads as w0 sqrt(1 + (z/z_R)^2),
    z_R = pi w0^2 n0 / lambda (paraxial error ~ 1/(k w0)^2 ~ 1e-3)."""
    n, dx, dz, lam, n0, w0, steps = 256, 0.2, 0.2, 0.5, 1.33, 2.0, 100
    xs = synth.lateral_coords(n, dx)
    r2 = xs[None, :] ** 2 + xs[:, None] ** 2
    u0 = np.exp(-r2 / w0 ** 2)
    u, _ = oracle.bpm_forward(u0, np.zeros((steps, n, n)), dx, dz, lam, n0, intensity=False)
    i2 = np.abs(u) ** 2
    w_meas = 2 * np.sqrt((xs[None, :] ** 2 * i2).sum() / i2.sum())
    z_r = np.pi * w0 ** 2 * n0 / lam
    w_theory = w0 * np.sqrt(1 + (steps * dz / z_r) ** 2)
    assert abs(w_meas / w_theory - 1) < 5e-3


def test_defocused_point_source_focuses_at_depth():
    """The source of the plain workload (focus 2 um downstream, dz = 0.1 um)
    has its on-axis intensity maximum at slice 2 / 0.1 - 1 = 19 in dn = 0."""
    g = synth.Geometry(128, 128, 40, 0.1, 0.1)
    u0 = synth.point_source_field(g.nx, g.ny, g.dx, g.wavelength, g.n0, 0.6, 2.0)
    _, inten = oracle.bpm_forward(u0, np.zeros((g.steps, g.ny, g.nx)), g.dx, g.dz,
                                  g.wavelength, g.n0)
    axis = inten[:, g.ny // 2, g.nx // 2]
    assert abs(int(np.argmax(axis)) - 19) <= 1


# ---------------------------------------------------------------------------
# whole recursion against explicit matrices

def test_tiny_dense_recursion():
    """8 x 4 grid, 3 steps: u <- S_j (F^-1 diag(H) F u) with F built from
    exp(-2 pi i n k / N) matrices and H from the dispersion relation."""
    nx, ny, steps, dx, dz, lam, n0 = 8, 4, 3, 0.11, 0.17, 0.5, 1.33
    rng = np.random.default_rng(8)
    u0 = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    dn = rng.uniform(-0.05, 0.05, (steps, ny, nx))
    fx = np.exp(-2j * np.pi * np.outer(np.arange(nx), np.arange(nx)) / nx)
    fy = np.exp(-2j * np.pi * np.outer(np.arange(ny), np.arange(ny)) / ny)
    m = np.where(np.arange(nx) < nx // 2, np.arange(nx), np.arange(nx) - nx)
    l = np.where(np.arange(ny) < ny // 2, np.arange(ny), np.arange(ny) - ny)
    kz = kz_of(m[None, :], l[:, None], nx, ny, dx, lam, n0)
    h = np.where(np.imag(kz) == 0, np.exp(1j * dz * np.real(kz)), 0)
    assert 0 < (h == 0).sum() < h.size            # both kinds of mode present
    u = u0.copy()
    for j in range(steps):
        spec = fy @ u @ fx.T
        u = np.linalg.inv(fy) @ (h * spec) @ np.linalg.inv(fx.T)
        u = np.exp(1j * TWO_PI / lam * dz * dn[j]) * u
    got, inten = oracle.bpm_forward(u0, dn, dx, dz, lam, n0)
    assert np.abs(got - u).max() <= 1e-13
    assert np.abs(inten[-1] - np.abs(u) ** 2).max() <= 1e-13


# ---------------------------------------------------------------------------
# multiplexing and statelessness

def test_linearity_is_multiplexing():
    """march(a u1 + b u2) = a march(u1) + b march(u2): independent sources
    can share one field."""
    g = synth.Geometry(64, 64, 12, 0.2, 0.2)
    rng = np.random.default_rng(9)
    dn = rng.uniform(0, 0.05, (g.steps, g.ny, g.nx))
    u1 = synth.point_source_field(64, 64, 0.2, 0.5, 1.33, 0.6, 1.0, centre=(16, 16)).astype(complex)
    u2 = synth.point_source_field(64, 64, 0.2, 0.5, 1.33, 0.6, 1.0, centre=(40, 48)).astype(complex)
    a, b = 0.3 - 0.8j, 1.1 + 0.2j
    lhs, _ = oracle.bpm_forward(a * u1 + b * u2, dn, g.dx, g.dz, 0.5, 1.33)
    r1, _ = oracle.bpm_forward(u1, dn, g.dx, g.dz, 0.5, 1.33)
    r2, _ = oracle.bpm_forward(u2, dn, g.dx, g.dz, 0.5, 1.33)
    assert rel(lhs, a * r1 + b * r2) <= 1e-13


def test_resume_is_bitwise():
    """N steps equal k steps followed by N - k steps, bit for bit."""
    rng = np.random.default_rng(10)
    u0 = rng.standard_normal((32, 64)) + 1j * rng.standard_normal((32, 64))
    dn = rng.uniform(0, 0.05, (10, 32, 64))
    full, inten = oracle.bpm_forward(u0, dn, 0.2, 0.2, 0.5, 1.33)
    half, i1 = oracle.bpm_forward(u0, dn[:4], 0.2, 0.2, 0.5, 1.33)
    rest, i2 = oracle.bpm_forward(half, dn[4:], 0.2, 0.2, 0.5, 1.33)
    assert np.array_equal(full, rest)
    assert np.array_equal(inten, np.concatenate([i1, i2]))


def test_zero_steps_is_identity():
    u0 = np.arange(32 * 32).reshape(32, 32) * (1 + 1j)
    u, inten = oracle.bpm_forward(u0, np.zeros((0, 32, 32)), 0.2, 0.2, 0.5, 1.33)
    assert np.array_equal(u, u0) and inten.shape == (0, 32, 32)


def test_staggered_start_equals_marching_from_depth():
    """A source that enters the march k slices early as the clear-medium
    field focusing k dz downstream, with the first k screens skipped (dn = 0
    there), leaves the volume exactly as the in-focus source marched from
    slice k: free-space steps compose (H^k applied to exp(-i kz k dz))."""
    n, N, k = 64, 12, 5
    rng = np.random.default_rng(11)
    dn = rng.uniform(0, 0.05, (N, n, n))
    src = [[20, 30], [45, 12]]
    focused = oracle.point_sources(n, n, 0.2, 0.5, 1.33, 0.6, 0.0, src)
    early = oracle.point_sources(n, n, 0.2, 0.5, 1.33, 0.6, k * 0.2, src)
    cleared = dn.copy()
    cleared[:k] = 0.0
    a, _ = oracle.bpm_forward(early, cleared, 0.2, 0.2, 0.5, 1.33, intensity=False)
    b, _ = oracle.bpm_forward(focused, dn[k:], 0.2, 0.2, 0.5, 1.33, intensity=False)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
