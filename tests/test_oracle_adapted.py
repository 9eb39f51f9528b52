"""Pins of the oracle's locally adapted expansion (per-slice reference index,
oracle_bpm_forward_adapted).

* dn_ref = 0 reduces to the plain march (already pinned), bit for bit;
* a plane wave through homogeneous layers n0 + c_j, each expanded about its
  own index, picks up exactly the layered-medium phase
  dz sum_j sqrt(((n0 + c_j) k0)^2 - kt^2) (closed form: the transverse
  wavenumber is conserved and each layer is a homogeneous medium), while the
  plain expansion about n0 deviates by the known amount;
* a mode with (n0 k0)^2 < kt^2 <= ((n0 + c) k0)^2 propagates with unit
  modulus when the slice is expanded about n0 + c and is cut to zero when it
  is expanded about n0;
* energy is non-increasing with a random reference index per slice.
"""
import numpy as np

import oracle

LAM, N0 = 0.5, 1.33


def plane_wave(nx, ny, qx, qy):
    y, x = np.mgrid[0:ny, 0:nx]
    return np.exp(2j * np.pi * (qx * x / nx + qy * y / ny))


def test_zero_reference_is_the_plain_march():
    rng = np.random.default_rng(1)
    u0 = rng.standard_normal((32, 64)) + 1j * rng.standard_normal((32, 64))
    dn = rng.uniform(0, 0.05, (5, 32, 64))
    a, ia = oracle.bpm_forward(u0, dn, 0.2, 0.2, LAM, N0)
    b, ib = oracle.bpm_forward_adapted(u0, dn, np.zeros(5), 0.2, 0.2, LAM, N0)
    assert np.array_equal(a, b) and np.array_equal(ia, ib)


def test_layered_medium_phase_of_a_plane_wave():
    nx = ny = 64
    dx = dz = 0.2
    qx, qy = 9, -5
    c = np.array([0.0, 0.03, 0.01, 0.05, 0.02, 0.04])
    dn = np.broadcast_to(c[:, None, None], (len(c), ny, nx)).copy()
    u0 = plane_wave(nx, ny, qx, qy)
    k0 = 2 * np.pi / LAM
    kt2 = (2 * np.pi * qx / (nx * dx)) ** 2 + (2 * np.pi * qy / (ny * dx)) ** 2
    exact = dz * np.sum(np.sqrt(((N0 + c) * k0) ** 2 - kt2))
    plain = dz * np.sum(np.sqrt((N0 * k0) ** 2 - kt2) + k0 * c)
    ua, _ = oracle.bpm_forward_adapted(u0, dn, c, dx, dz, LAM, N0, intensity=False)
    up, _ = oracle.bpm_forward(u0, dn, dx, dz, LAM, N0, intensity=False)
    assert np.abs(ua - u0 * np.exp(1j * exact)).max() <= 1e-12
    assert np.abs(up - u0 * np.exp(1j * plain)).max() <= 1e-12
    assert abs(exact - plain) > 1e-3          # the two expansions differ for kt != 0


def test_adapted_evanescent_boundary():
    nx = ny = 128
    dx = dz = 0.2
    # propagating about n0: m~^2 + l~^2 <= (128 n0 dx / lambda)^2 = 68.1^2 = 4637;
    # about n0 + 0.05: <= 70.6^2 = 4992.  Mode (49, 48) (4705) lies between
    # the two cuts, mode (50, 50) (5000) beyond both.
    c = 0.05
    dn = np.full((3, ny, nx), c)
    ref = np.full(3, c)
    u0 = plane_wave(nx, ny, 49, 48)
    ua, _ = oracle.bpm_forward_adapted(u0, dn, ref, dx, dz, LAM, N0, intensity=False)
    up, _ = oracle.bpm_forward(u0, dn, dx, dz, LAM, N0, intensity=False)
    assert np.abs(np.abs(ua) - 1).max() <= 1e-12
    assert np.abs(up).max() <= 1e-12
    u_far = plane_wave(nx, ny, 50, 50)
    ua_far, _ = oracle.bpm_forward_adapted(u_far, dn, ref, dx, dz, LAM, N0, intensity=False)
    assert np.abs(ua_far).max() <= 1e-12


def test_energy_non_increasing_with_random_references():
    rng = np.random.default_rng(4)
    u0 = rng.standard_normal((64, 64)) + 1j * rng.standard_normal((64, 64))
    dn = rng.uniform(0, 0.05, (6, 64, 64))
    ref = rng.uniform(-0.02, 0.06, 6)
    _, inten = oracle.bpm_forward_adapted(u0, dn, ref, 0.2, 0.2, LAM, N0)
    e = np.concatenate([[np.sum(np.abs(u0) ** 2)], inten.sum(axis=(1, 2))])
    assert np.all(np.diff(e) <= 1e-10 * e[0])
    # every mode propagating (dx = 0.3 um > lambda / (sqrt 2 n_min)): conserved
    _, inten3 = oracle.bpm_forward_adapted(u0, dn, np.abs(ref), 0.3, 0.2, LAM, N0)
    e3 = inten3.sum(axis=(1, 2))
    assert np.abs(e3 / e[0] - 1).max() <= 1e-12
