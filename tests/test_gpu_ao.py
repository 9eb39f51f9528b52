"""GPU parity of the adaptive-optics path (linear adjoint, guide-star phase,
pupil optimiser, memory effect) with the FP64 oracle.

* the linear adjoint (field_in NULL, no intensity or dn gradient) against the
  oracle adjoint and bitwise against the full adjoint of the same gradient;
* the guide-star phase kernel against its closed form, incl. the shift tilt;
* on the Perlin tissue (256^2 x 80, n = 1.36 +- 0.03, about four mean free
  paths): the corrected and aimed focus intensities against the oracle, the
  corrected intensity at the Cauchy-Schwarz optimum (sum A |G|)^2;
* the multi-focus phase gradient against the oracle, and Adam from the aimed
  phase reaching the guide-star optimum;
* memory-effect persistence, plane-wave speckle autocorrelation and mean free
  paths against the oracle, and the persistence range against the speckle
  correlation length.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import ao as oao

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def to_gpu(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype)).cuda()


def cpu(t):
    return t.cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("nx,ny,steps", [(64, 128, 10), (256, 256, 33), (1024, 64, 6),
                                         (32, 64, 1), (64, 32, 0)])
def test_linear_adjoint(nx, ny, steps):
    import paper_1706_02261_amd as bpm
    rng = np.random.default_rng(nx + 3 * ny + steps)
    w = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
    u0 = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
    dn = rng.uniform(-0.03, 0.03, (steps, ny, nx)).astype(np.float32)
    dn_t, w_t = to_gpu(dn, np.float32), to_gpu(w, np.complex64)
    g0, gs, gdn = bpm.adjoint(None, dn_t, 0.2, 0.2, 0.5, 1.36, grad_field_out=w_t,
                              want_spectrum=True, want_dn=False)
    assert gdn is None
    r0, rs, _ = oracle.bpm_adjoint(np.zeros((ny, nx), complex), dn, 0.2, 0.2, 0.5, 1.36,
                                   grad_u_out=w)
    assert rel(cpu(g0), r0) <= 2e-5 and rel(cpu(gs), rs) <= 2e-5
    # the full adjoint (forward march, checkpoints, dn gradient) gives the same bits
    f0, fs, _ = bpm.adjoint(to_gpu(u0, np.complex64), dn_t, 0.2, 0.2, 0.5, 1.36,
                            grad_field_out=w_t, want_spectrum=True, want_dn=True)
    torch.cuda.synchronize()
    assert np.array_equal(cpu(f0), cpu(g0)) and np.array_equal(cpu(fs), cpu(gs))


def test_linear_adjoint_needs_field_for_other_gradients():
    import paper_1706_02261_amd as bpm
    dn = torch.zeros((3, 64, 64), dtype=torch.float32, device="cuda")
    w = torch.zeros((64, 64), dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError):
        bpm.adjoint(None, dn, 0.2, 0.2, 0.5, 1.36, grad_field_out=w, want_dn=True)


@pytest.mark.parametrize("shift", [(0.0, 0.0), (0.6, -1.4), (-3.0, 2.2)])
def test_guide_star_phase_kernel(shift):
    import paper_1706_02261_amd as bpm
    rng = np.random.default_rng(7)
    nx, ny, zf = 256, 128, 16.0
    G = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
    got = cpu(bpm.guide_star_phase(to_gpu(G, np.complex64), 0.2, 0.5, 1.36, zf, shift=shift))
    ref = oao.guide_star_phase(G.astype(complex), 0.2, 0.5, 1.36, zf, shift=shift)
    assert got.min() >= -np.pi and got.max() <= np.pi
    assert np.abs(oao.wrap(got - ref)).max() <= 2e-6


# ---------------------------------------------------------------------------
# the Perlin tissue

@pytest.fixture(scope="module")
def tissue():
    g, dn, amp, zf = synth.ao_workload(256, 80)
    focus = (g.ny // 2, g.nx // 2)
    dn64 = dn.astype(float)
    gs_o = oao.guide_star_gradient(dn64, focus, g.dx, g.dz, g.wavelength, g.n0)
    return dict(g=g, dn=dn, dn64=dn64, amp=amp, zf=zf, focus=focus, gs_o=gs_o,
                dn_t=to_gpu(dn, np.float32), amp_t=to_gpu(amp, np.float32))


def optics_of(g):
    from paper_1706_02261_amd import ao
    return ao.Optics(g.dx, g.dz, g.wavelength, g.n0)


def test_guide_star_correction(tissue):
    from paper_1706_02261_amd import ao
    g, f, zf = tissue["g"], tissue["focus"], tissue["zf"]
    opt = optics_of(g)
    phi, gs = ao.guide_star_phase(tissue["dn_t"], f, zf, opt)
    assert rel(cpu(gs), tissue["gs_o"]) <= 2e-5
    best = oao.optimum_intensity(tissue["amp"], tissue["gs_o"])
    inten = cpu(ao.exit_field(tissue["amp_t"], phi, tissue["dn_t"], zf, opt).abs() ** 2)
    aim = ao.aim_phase(g.ny, g.nx, f, opt)
    unc = cpu(ao.exit_field(tissue["amp_t"], aim, tissue["dn_t"], zf, opt).abs() ** 2)
    clear = cpu(ao.exit_field(tissue["amp_t"], aim, torch.zeros_like(tissue["dn_t"]), zf,
                              opt).abs() ** 2)
    unc_o = abs(oao.exit_field(tissue["amp"], oao.aim_phase(g.nx, g.ny, g.dx, g.wavelength, g.n0,
                                                            f),
                               tissue["dn64"], g.dx, g.dz, g.wavelength, g.n0, zf)[f]) ** 2
    print(f"focus: clear {clear[f]:.4e} aimed {unc[f]:.4e} corrected {inten[f]:.4e} "
          f"optimum {best:.4e}")
    assert abs(inten[f] / best - 1) <= 1e-4
    assert abs(unc[f] / unc_o - 1) <= 1e-4
    assert np.unravel_index(np.argmax(inten), inten.shape) == f
    assert inten[f] >= 4 * unc[f] and inten[f] >= 0.5 * clear[f]


def test_guide_star_gradients_of_several_foci(tissue):
    """Ten guide stars (two lockstep launches of 8 and 2): bitwise the single
    adjoints, and the oracle's G for two of them."""
    from paper_1706_02261_amd import ao
    g = tissue["g"]
    opt = optics_of(g)
    foci = [(100 + 6 * k, 90 + 9 * k) for k in range(10)]
    many = ao.guide_star_gradients(tissue["dn_t"], foci, opt)
    assert len(many) == len(foci)
    for f, gs in zip(foci, many):
        assert torch.equal(gs, ao.guide_star_gradient(tissue["dn_t"], f, opt))
    for k in (0, 9):
        ref = oao.guide_star_gradient(tissue["dn64"], foci[k], g.dx, g.dz, g.wavelength, g.n0)
        assert rel(cpu(many[k]), ref) <= 2e-5


def test_focus_gradient_two_foci(tissue):
    from paper_1706_02261_amd import ao
    g, zf = tissue["g"], tissue["zf"]
    opt = optics_of(g)
    foci = [(128, 128), (120, 141)]
    rng = np.random.default_rng(8)
    phi = rng.uniform(-np.pi, np.pi, (g.ny, g.nx)).astype(np.float32)
    inten, gphi = ao.focus_gradient(tissue["amp_t"], to_gpu(phi, np.float32), tissue["dn_t"],
                                    foci, zf, opt)
    # oracle: L = -sum |u_f|^2, dL/dU0 = sum_f -2 u_f G_f, dL/dphi = Im(dL/dU0 conj(U0))
    u = oao.exit_field(tissue["amp"], phi, tissue["dn64"], g.dx, g.dz, g.wavelength, g.n0, zf)
    U0 = oao.pupil_spectrum(tissue["amp"], phi, g.dx, g.wavelength, g.n0, zf)
    G = sum(-2 * u[f] * oao.guide_star_gradient(tissue["dn64"], f, g.dx, g.dz, g.wavelength,
                                                g.n0) for f in foci)
    ref = np.imag(G * np.conj(U0))
    assert rel(cpu(gphi), ref) <= 1e-4
    assert np.abs(cpu(inten) / np.array([abs(u[f]) ** 2 for f in foci]) - 1).max() <= 1e-4


def test_adam_optimizer_reaches_the_guide_star_optimum(tissue):
    from paper_1706_02261_amd import ao
    g, f, zf = tissue["g"], tissue["focus"], tissue["zf"]
    opt = optics_of(g)
    best = oao.optimum_intensity(tissue["amp"], tissue["gs_o"])
    aim = ao.aim_phase(g.ny, g.nx, f, opt)
    phase, hist = ao.optimize_pupil(tissue["amp_t"], tissue["dn_t"], [f], zf, opt, iters=60,
                                    lr=0.1, phase0=aim)
    h = cpu(hist)[:, 0] / best
    final = float(cpu(ao.exit_field(tissue["amp_t"], phase, tissue["dn_t"], zf, opt)[f].abs())
                  ** 2) / best
    print("fraction of the optimum by iteration:", np.round(h[[0, 4, 9, 19, 39, 59]], 4), final)
    assert h[0] < 0.5 and final >= 0.99 and final <= 1 + 1e-4


def test_adam_step_matches_the_oracle():
    import paper_1706_02261_amd as bpm
    from oracle import surrogate_net
    rng = np.random.default_rng(9)
    n = 5000
    w = rng.standard_normal(n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    wt, mt, vt = to_gpu(w, np.float32), to_gpu(m, np.float32), to_gpu(v, np.float32)
    w64, m64, v64 = w.astype(float), m.astype(float), v.astype(float)
    for t in range(1, 4):
        gr = rng.standard_normal(n).astype(np.float32)
        bpm.adam_step(wt, to_gpu(gr, np.float32), mt, vt, 0.01, t)
        w64, m64, v64 = surrogate_net.adam_step(w64, gr.astype(float), m64, v64, t, 0.01)
    assert np.abs(cpu(wt) - w64).max() <= 2e-6 and rel(cpu(mt), m64) <= 1e-6


def test_memory_effect_and_speckle(tissue):
    from paper_1706_02261_amd import ao
    g, f, zf = tissue["g"], tissue["focus"], tissue["zf"]
    opt = optics_of(g)
    shifts = [(0, 1), (0, 2), (0, 3), (0, 4), (0, 6), (1, 0), (2, 0), (3, 0), (4, 0), (6, 0),
              (-3, 5)]
    _, gs = ao.guide_star_phase(tissue["dn_t"], f, zf, opt)
    P, base = ao.memory_effect(tissue["amp_t"], gs, tissue["dn_t"], f, shifts, zf, opt)
    P_o, base_o = oao.memory_effect(tissue["amp"], tissue["gs_o"], tissue["dn64"], f, shifts,
                                    g.dx, g.dz, g.wavelength, g.n0, zf)
    print("P", np.round(P, 4), "oracle", np.round(P_o, 4))
    assert abs(base / base_o - 1) <= 1e-4 and np.abs(P - P_o).max() <= 2e-4
    pw = ao.plane_wave_exit(tissue["dn_t"], opt)
    C = ao.speckle_autocorrelation((pw.abs() ** 2).contiguous(), 8)
    pw_o = oao.plane_wave_speckle(tissue["dn64"], g.dx, g.dz, g.wavelength, g.n0)
    C_o = oao.speckle_autocorrelation(np.abs(pw_o) ** 2, 8)
    mfp, mfp_o = ao.mean_free_paths(pw), oao.mean_free_paths(pw_o)
    print("C", np.round(C, 4), "mfp", mfp, mfp_o)
    assert np.abs(C - C_o).max() <= 1e-4 and abs(mfp - mfp_o) <= 1e-3
    assert 3.0 <= mfp <= 6.0

    def half_width(c):
        for i in range(1, len(c)):
            if c[i] < 0.5:
                return i - 1 + (c[i - 1] - 0.5) / (c[i - 1] - c[i])
        return float("inf")
    Pm = np.r_[1.0, 0.5 * (P[:4] + P[5:9])]
    assert abs(half_width(Pm) / half_width(C[:5]) - 1) <= 0.25


def test_edge_cases():
    """No shifts, no ballistic light, a zero-step tissue."""
    from paper_1706_02261_amd import ao
    g, dn, amp, zf = synth.ao_workload(64, 4)
    opt = ao.Optics(g.dx, g.dz, g.wavelength, g.n0)
    dn_t, amp_t = to_gpu(dn, np.float32), to_gpu(amp, np.float32)
    _, gs = ao.guide_star_phase(dn_t, (32, 32), zf, opt)
    P, base = ao.memory_effect(amp_t, gs, dn_t, (32, 32), [], zf, opt)
    assert P.shape == (0,) and base > 0
    assert ao.mean_free_paths(torch.zeros((8, 8), dtype=torch.complex64, device="cuda")) == float("inf")
    # zero steps: the guide-star phase of an empty tissue is the aiming tilt of a focus at z_f
    phi0, _ = ao.guide_star_phase(dn_t[:0], (5, 9), 0.0, opt)
    aim = ao.aim_phase(64, 64, (5, 9), opt)
    diff = oao.wrap(cpu(phi0).astype(float) - cpu(aim).astype(float))
    assert np.abs(diff[amp > 0]).max() <= 1e-5
