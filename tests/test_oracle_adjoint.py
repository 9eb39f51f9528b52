"""Pins of the oracle's adjoint march.

* dot-product test: the backward map is the Hermitian adjoint of the forward;
* central finite differences of the forward oracle (h = 1e-3);
* phase conjugation (guide-star adaptive optics): the conjugated pupil reaches
  the Cauchy-Schwarz bound and is a stationary point;
* gauge invariance: a constant added to one slice only changes a global phase.
"""
import numpy as np
import pytest

import oracle
import synth

LAM, N0 = 0.5, 1.33


def rand_c(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_dot_product():
    """<w, M u> = <M^H w, u> for random u, w and random dn."""
    rng = np.random.default_rng(11)
    ny, nx, steps = 16, 32, 5
    u, w = rand_c(rng, (ny, nx)), rand_c(rng, (ny, nx))
    dn = rng.uniform(0, 0.06, (steps, ny, nx))
    mu, _ = oracle.bpm_forward(u, dn, 0.1, 0.2, LAM, N0, intensity=False)
    mhw, _, _ = oracle.bpm_adjoint(u, dn, 0.1, 0.2, LAM, N0, grad_u_out=w)
    lhs = np.vdot(w, mu)
    rhs = np.vdot(mhw, u)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def pupil_setup(nxy=32, steps=10, seed=12):
    g, dn, amp, z_f = synth.config3(steps=steps, nxy=nxy)
    rng = np.random.default_rng(seed)
    dn = dn + rng.uniform(0, 0.02, dn.shape)        # make every voxel matter
    k = N0 * 2 * np.pi / LAM
    kx = 2 * np.pi * np.fft.fftfreq(g.nx, d=g.dx)[None, :]
    ky = 2 * np.pi * np.fft.fftfreq(g.ny, d=g.dx)[:, None]
    kz = np.sqrt(np.maximum(k * k - kx ** 2 - ky ** 2, 0))
    return g, dn, amp, kz, z_f


def field_of(amp, phi, kz, z_f):
    """u0 = IDFT2(A exp(i phi) exp(-i kz z_f)) (numpy's ifft2 as the library step)."""
    return np.fft.ifft2(amp * np.exp(1j * phi) * np.exp(-1j * kz * z_f))


def focal_loss(g, dn, u0, jf, yf, xf):
    _, inten = oracle.bpm_forward(u0, dn, g.dx, g.dz, LAM, N0)
    return -inten[jf, yf, xf]


def test_finite_differences_pupil_and_dn():
    """Loss = -I[j_f][centre]; gradients in phi (pupil) and dn vs central
    differences with h = 1e-3 on random coordinates."""
    g, dn, amp, kz, z_f = pupil_setup()
    rng = np.random.default_rng(13)
    phi = rng.uniform(0, 2 * np.pi, amp.shape)
    jf, yf, xf = g.steps - 1, g.ny // 2, g.nx // 2
    u0 = field_of(amp, phi, kz, z_f)
    gi = np.zeros((g.steps, g.ny, g.nx))
    gi[jf, yf, xf] = -1.0
    _, gspec, gdn = oracle.bpm_adjoint(u0, dn, g.dx, g.dz, LAM, N0, grad_intensity=gi)
    u_spec = amp * np.exp(1j * phi) * np.exp(-1j * kz * z_f)
    gphi = np.imag(gspec * np.conj(u_spec))
    h = 1e-3
    scale_phi = np.abs(gphi).max()
    support = np.argwhere(amp > 0.05)
    for idx in support[rng.choice(len(support), 12, replace=False)]:
        p1, p2 = phi.copy(), phi.copy()
        p1[tuple(idx)] += h
        p2[tuple(idx)] -= h
        fd = (focal_loss(g, dn, field_of(amp, p1, kz, z_f), jf, yf, xf)
              - focal_loss(g, dn, field_of(amp, p2, kz, z_f), jf, yf, xf)) / (2 * h)
        assert abs(gphi[tuple(idx)] - fd) <= 1e-4 * max(abs(fd), 1e-2 * scale_phi)
    scale_dn = np.abs(gdn).max()
    for _ in range(12):
        idx = (rng.integers(0, jf), rng.integers(0, g.ny), rng.integers(0, g.nx))
        d1, d2 = dn.copy(), dn.copy()
        d1[idx] += h
        d2[idx] -= h
        fd = (focal_loss(g, d1, u0, jf, yf, xf) - focal_loss(g, d2, u0, jf, yf, xf)) / (2 * h)
        assert abs(gdn[idx] - fd) <= 1e-4 * max(abs(fd), 1e-2 * scale_dn)


def test_field_gradient_finite_differences():
    """Loss = Re<w, u_N> + sum c I: gradient w.r.t. Re/Im of u0 vs differences."""
    rng = np.random.default_rng(14)
    ny, nx, steps = 16, 16, 4
    u0, w = rand_c(rng, (ny, nx)), rand_c(rng, (ny, nx))
    dn = rng.uniform(0, 0.05, (steps, ny, nx))
    cI = rng.standard_normal((steps, ny, nx))

    def loss(u):
        out, inten = oracle.bpm_forward(u, dn, 0.2, 0.2, LAM, N0)
        return np.real(np.vdot(w, out)) + np.sum(cI * inten)

    g0, _, _ = oracle.bpm_adjoint(u0, dn, 0.2, 0.2, LAM, N0, grad_u_out=w, grad_intensity=cI)
    h = 1e-4
    for _ in range(8):
        iy, ix = rng.integers(0, ny), rng.integers(0, nx)
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            a, b = u0.copy(), u0.copy()
            a[iy, ix] += unit * h
            b[iy, ix] -= unit * h
            fd = (loss(a) - loss(b)) / (2 * h)
            assert abs(part(g0[iy, ix]) - fd) <= 1e-6 * max(1.0, abs(fd))


def test_phase_conjugation_optimum():
    """Guide star: c = conj(DFT(M^H e_f)) / N gives u_N(x_f) = sum_k c_k U0_k.
    phi* = arg(DFT(M^H e_f)) + kz z_f makes every term real positive, so
    L(phi*) = -(sum A |c|)^2, the gradient vanishes and random pupils do worse."""
    g, dn, amp, kz, z_f = pupil_setup(seed=15)
    n = g.nx * g.ny
    yf, xf = g.ny // 2, g.nx // 2
    ef = np.zeros((g.ny, g.nx), complex)
    ef[yf, xf] = 1.0
    mh_ef, _, _ = oracle.bpm_adjoint(np.zeros_like(ef), dn, g.dx, g.dz, LAM, N0, grad_u_out=ef)
    d = np.fft.fft2(mh_ef)
    c = np.conj(d) / n
    phi_star = np.angle(d) + kz * z_f
    bound = (amp * np.abs(c)).sum() ** 2
    u0 = field_of(amp, phi_star, kz, z_f)
    out, _ = oracle.bpm_forward(u0, dn, g.dx, g.dz, LAM, N0, intensity=False)
    loss_star = -abs(out[yf, xf]) ** 2
    assert abs(loss_star + bound) <= 1e-10 * bound
    # stationary point of L(phi) = -|u_N(x_f)|^2
    gout = -2 * out[yf, xf] * ef
    _, gspec, _ = oracle.bpm_adjoint(u0, dn, g.dx, g.dz, LAM, N0, grad_u_out=gout)
    u_spec = amp * np.exp(1j * phi_star) * np.exp(-1j * kz * z_f)
    gphi = np.imag(gspec * np.conj(u_spec))
    assert np.abs(gphi).max() <= 1e-10 * bound
    rng = np.random.default_rng(16)
    for _ in range(3):
        u_r = field_of(amp, rng.uniform(0, 2 * np.pi, amp.shape), kz, z_f)
        o_r, _ = oracle.bpm_forward(u_r, dn, g.dx, g.dz, LAM, N0, intensity=False)
        assert -abs(o_r[yf, xf]) ** 2 >= loss_star


def test_gauge_invariance_of_dn_gradient():
    """For a loss of |u| only: each slice's dn gradient sums to zero; slices
    at and after the loss slice have zero gradient."""
    rng = np.random.default_rng(17)
    ny, nx, steps, jf = 32, 32, 8, 5
    u0 = rand_c(rng, (ny, nx))
    dn = rng.uniform(0, 0.05, (steps, ny, nx))
    gi = np.zeros((steps, ny, nx))
    gi[jf] = rng.standard_normal((ny, nx))
    _, _, gdn = oracle.bpm_adjoint(u0, dn, 0.2, 0.2, LAM, N0, grad_intensity=gi)
    l1 = np.abs(gdn).sum()
    assert np.abs(gdn.sum(axis=(1, 2))).max() <= 1e-12 * l1
    assert np.abs(gdn[:jf]).max() > 0
    assert np.abs(gdn[jf:]).max() <= 1e-13 * np.abs(gdn[:jf]).max()


@pytest.mark.parametrize("steps", [0, 1])
def test_tiny_step_counts(steps):
    rng = np.random.default_rng(18)
    u0, w = rand_c(rng, (8, 8)), rand_c(rng, (8, 8))
    dn = rng.uniform(0, 0.05, (steps, 8, 8))
    g0, gs, gdn = oracle.bpm_adjoint(u0, dn, 0.2, 0.2, LAM, N0, grad_u_out=w)
    if steps == 0:
        assert np.array_equal(g0, w) and gdn.shape == (0, 8, 8)
    mu, _ = oracle.bpm_forward(u0, dn, 0.2, 0.2, LAM, N0)
    assert abs(np.vdot(w, mu) - np.vdot(g0, u0)) <= 1e-12 * abs(np.vdot(w, mu))
    assert np.abs(gs - np.fft.fft2(g0) / 64).max() <= 1e-13
