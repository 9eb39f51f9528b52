"""GPU parity of the adjoint march (bpm_adjoint) and its helpers.

* element-wise parity of dL/du0, dL/dU0 and dL/ddn with the FP64 oracle;
* checkpoint interval invariance (bitwise) and the dot-product test;
* the adaptive-optics workload (256^2 x 512, pupil phase and dn gradients of
  the negative focal intensity) against the oracle gradient and against
  central finite differences (h = 1e-3) evaluated in the FP64 oracle;
* the natural-order 2-D FFT and the pupil-plane helpers.
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


def to_gpu(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype)).cuda()


def cpu(t):
    return None if t is None else t.cpu().numpy()


def rand_case(nx, ny, steps, seed):
    rng = np.random.default_rng(seed)
    u0 = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
    w = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
    gI = rng.standard_normal((steps, ny, nx)).astype(np.float32)
    dn = rng.uniform(0, 0.05, (steps, ny, nx)).astype(np.float32)
    return u0, w, gI, dn


def gpu_adjoint(u0, dn, w, gI, dx=0.2, dz=0.2, ck=0):
    import paper_1706_02261_amd as bpm
    g0, gs, gdn = bpm.adjoint(to_gpu(u0, np.complex64), to_gpu(dn, np.float32), dx, dz, LAM, N0,
                              grad_field_out=None if w is None else to_gpu(w, np.complex64),
                              grad_intensity=None if gI is None else to_gpu(gI, np.float32),
                              want_spectrum=True, checkpoint_every=ck)
    torch.cuda.synchronize()
    return cpu(g0), cpu(gs), cpu(gdn)


@pytest.mark.parametrize("nx,ny,steps", [(64, 128, 10), (128, 32, 7), (256, 256, 33), (32, 64, 1),
                                         (1024, 64, 6), (64, 1024, 5)])
def test_adjoint_parity(nx, ny, steps):
    """Oracle gradients; sides above 512 take the 256-thread-workgroup kernel."""
    u0, w, gI, dn = rand_case(nx, ny, steps, seed=nx + ny + steps)
    g0, gs, gdn = gpu_adjoint(u0, dn, w, gI)
    r0, rs, rdn = oracle.bpm_adjoint(u0, dn, 0.2, 0.2, LAM, N0, grad_u_out=w, grad_intensity=gI)
    print(f"g0 {rel(g0, r0):.2e} spectrum {rel(gs, rs):.2e} dn {rel(gdn, rdn):.2e}")
    assert rel(g0, r0) <= 2e-5 and rel(gs, rs) <= 2e-5 and rel(gdn, rdn) <= 2e-5


@pytest.mark.parametrize("which", ["field", "intensity"])
def test_adjoint_single_source_of_gradient(which):
    u0, w, gI, dn = rand_case(64, 64, 6, seed=4)
    w, gI = (w, None) if which == "field" else (None, gI)
    g0, gs, gdn = gpu_adjoint(u0, dn, w, gI)
    r0, rs, rdn = oracle.bpm_adjoint(u0, dn, 0.2, 0.2, LAM, N0, grad_u_out=w, grad_intensity=gI)
    assert rel(g0, r0) <= 2e-5 and rel(gs, rs) <= 2e-5 and rel(gdn, rdn) <= 2e-5


def test_adjoint_zero_steps():
    u0, w, _, _ = rand_case(64, 32, 0, seed=5)
    g0, gs, gdn = gpu_adjoint(u0, np.zeros((0, 32, 64), np.float32), w, None)
    assert np.array_equal(g0, w) and gdn.shape == (0, 32, 64)
    assert rel(gs, np.fft.fft2(w.astype(complex)) / w.size) <= 1e-6


@pytest.mark.parametrize("nx,ny,steps", [(128, 128, 20), (1024, 64, 10)])
def test_checkpoint_interval_is_bitwise_invariant(nx, ny, steps):
    """Every checkpoint interval, including a shorter last segment and a
    single segment, gives the same bits."""
    u0, w, gI, dn = rand_case(nx, ny, steps, seed=6)
    ref = gpu_adjoint(u0, dn, w, gI, ck=0)
    for ck in sorted({1, 3, 7, steps}):
        got = gpu_adjoint(u0, dn, w, gI, ck=ck)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), f"checkpoint_every={ck}"


def test_dot_product_on_gpu():
    """<w, M u> = <M^H w, u> with the GPU forward and adjoint marches."""
    import paper_1706_02261_amd as bpm
    u0, w, _, dn = rand_case(256, 128, 12, seed=7)
    out, _ = bpm.propagate(to_gpu(u0, np.complex64), to_gpu(dn, np.float32), 0.2, 0.2, LAM, N0,
                           intensity=False)
    g0, _, _ = gpu_adjoint(u0, dn, w, None)
    lhs = np.vdot(w.astype(complex), cpu(out).astype(complex))
    rhs = np.vdot(g0.astype(complex), u0.astype(complex))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


# ---------------------------------------------------------------------------
# adaptive-optics workload: 256^2 x 512, loss = -I[N-1] at the grid centre

def ao_setup():
    g, dn, amp, z_f = synth.config3()
    phi = synth.rng(3, 1).uniform(0, 2 * np.pi, amp.shape)
    k = N0 * 2 * np.pi / LAM
    kx = 2 * np.pi * np.fft.fftfreq(g.nx, d=g.dx)[None, :]
    ky = 2 * np.pi * np.fft.fftfreq(g.ny, d=g.dx)[:, None]
    kz = np.sqrt(np.maximum(k * k - kx ** 2 - ky ** 2, 0))
    return g, dn, amp.astype(np.float32), phi.astype(np.float32), kz, z_f


def ao_field(amp, phi, kz, z_f):
    return np.fft.ifft2(amp.astype(float) * np.exp(1j * phi.astype(float)) * np.exp(-1j * kz * z_f))


@pytest.fixture(scope="module")
def ao():
    """GPU gradients (PupilBPMFunction) and the oracle's gradients of
    L = -I[N-1][centre] for the 256^2 x 512 sphere phantom."""
    import paper_1706_02261_amd as bpm
    g, dn, amp, phi, kz, z_f = ao_setup()
    jf, yf, xf = g.steps - 1, g.ny // 2, g.nx // 2
    phase = to_gpu(phi, np.float32).requires_grad_(True)
    dn_t = to_gpu(dn, np.float32).requires_grad_(True)
    out, inten = bpm.PupilBPMFunction.apply(phase, to_gpu(amp, np.float32), dn_t, g.dx, g.dz,
                                            LAM, N0, z_f)
    loss = -inten[jf, yf, xf]
    loss.backward()
    torch.cuda.synchronize()
    u0 = ao_field(amp, phi, kz, z_f)
    gi = np.zeros((g.steps, g.ny, g.nx))
    gi[jf, yf, xf] = -1.0
    _, rs, rdn = oracle.bpm_adjoint(u0, dn, g.dx, g.dz, LAM, N0, grad_intensity=gi)
    u_spec = amp * np.exp(1j * phi.astype(float)) * np.exp(-1j * kz * z_f)
    rphi = np.imag(rs * np.conj(u_spec))
    return dict(g=g, dn=dn, amp=amp, phi=phi, kz=kz, z_f=z_f, focus=(jf, yf, xf),
                gphi=cpu(phase.grad), gdn=cpu(dn_t.grad), rphi=rphi, rdn=rdn, u0=u0)


def test_adaptive_optics_gradient_vs_oracle(ao):
    e_phi, e_dn = rel(ao["gphi"], ao["rphi"]), rel(ao["gdn"], ao["rdn"])
    print(f"dphi rel err {e_phi:.2e}  ddn rel err {e_dn:.2e}")
    assert e_phi <= 1e-3 and e_dn <= 1e-3
    # gauge invariance: each slice's dn gradient sums to ~0, the loss slice's is 0
    jf = ao["focus"][0]
    l1 = np.abs(ao["gdn"]).sum()
    assert np.abs(ao["gdn"].sum(axis=(1, 2))).max() <= 1e-4 * l1
    assert np.abs(ao["gdn"][jf]).max() <= 1e-6 * np.abs(ao["gdn"]).max()


def _fd_ok(g_gpu, fd, scale):
    return abs(g_gpu - fd) <= 1e-3 * max(abs(fd), 1e-2 * scale)


def test_adaptive_optics_phase_finite_differences(ao):
    """Central differences (h = 1e-3) of the FP64 oracle at 32 seeded pupil
    coordinates inside the NA."""
    g, (jf, yf, xf) = ao["g"], ao["focus"]
    amp, kz, z_f, dn = ao["amp"], ao["kz"], ao["z_f"], ao["dn"]

    def loss(phi_):
        _, it = oracle.bpm_forward(ao_field(amp, phi_, kz, z_f), dn, g.dx, g.dz, LAM, N0)
        return -it[jf, yf, xf]

    rng = np.random.default_rng(33)
    support = np.argwhere(amp > 0.05)
    scale = np.abs(ao["rphi"]).max()
    for idx in support[rng.choice(len(support), 32, replace=False)]:
        p1, p2 = ao["phi"].astype(float), ao["phi"].astype(float)
        p1[tuple(idx)] += 1e-3
        p2[tuple(idx)] -= 1e-3
        fd = (loss(p1) - loss(p2)) / 2e-3
        assert _fd_ok(ao["gphi"][tuple(idx)], fd, scale), (tuple(idx), ao["gphi"][tuple(idx)], fd)


def test_adaptive_optics_dn_finite_differences(ao):
    """Central differences (h = 1e-3) of the FP64 oracle at 32 seeded dn voxels;
    each difference re-marches only the slices after the perturbed one."""
    g, (jf, yf, xf) = ao["g"], ao["focus"]
    dn = ao["dn"].astype(float)
    rng = np.random.default_rng(34)
    coords = sorted(((int(rng.integers(0, jf)), int(rng.integers(0, g.ny)),
                      int(rng.integers(0, g.nx))) for _ in range(32)))
    scale = np.abs(ao["rdn"]).max()
    u, at = ao["u0"], 0
    for (j, y, x) in coords:
        if j > at:
            u, _ = oracle.bpm_forward(u, dn[at:j], g.dx, g.dz, LAM, N0, intensity=False)
            at = j
        vals = []
        for h in (1e-3, -1e-3):
            tail = dn[j:].copy()
            tail[0, y, x] += h
            _, it = oracle.bpm_forward(u, tail, g.dx, g.dz, LAM, N0)
            vals.append(-it[jf - j, yf, xf])
        fd = (vals[0] - vals[1]) / 2e-3
        assert _fd_ok(ao["gdn"][j, y, x], fd, scale), ((j, y, x), ao["gdn"][j, y, x], fd)


def test_bpm_function_autograd_matches_oracle():
    import paper_1706_02261_amd as bpm
    u0, w, gI, dn = rand_case(128, 64, 9, seed=8)
    f = to_gpu(u0, np.complex64).requires_grad_(True)
    d = to_gpu(dn, np.float32).requires_grad_(True)
    out, inten = bpm.BPMFunction.apply(f, d, 0.2, 0.2, LAM, N0)
    loss = (torch.conj(to_gpu(w, np.complex64)) * out).real.sum() + (to_gpu(gI, np.float32) * inten).sum()
    loss.backward()
    r0, _, rdn = oracle.bpm_adjoint(u0, dn, 0.2, 0.2, LAM, N0, grad_u_out=w, grad_intensity=gI)
    assert rel(cpu(f.grad), r0) <= 2e-5 and rel(cpu(d.grad), rdn) <= 2e-5


# ---------------------------------------------------------------------------
# helpers

@pytest.mark.parametrize("nx,ny", [(32, 32), (64, 2048), (1024, 256)])
def test_fft2_natural_order(nx, ny):
    import paper_1706_02261_amd as bpm
    rng = np.random.default_rng(nx * ny)
    x = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
    fwd = cpu(bpm.fft2(to_gpu(x, np.complex64)))
    inv = cpu(bpm.fft2(to_gpu(x, np.complex64), inverse=True))
    assert rel(fwd, oracle.fft2d(x, -1)) <= 2e-6
    assert rel(inv, oracle.fft2d(x, +1) / x.size) <= 2e-6


def test_pupil_helpers():
    import paper_1706_02261_amd as bpm
    g, dn, amp, phi, kz, z_f = ao_setup()
    spec = cpu(bpm.pupil_spectrum(to_gpu(amp, np.float32), to_gpu(phi, np.float32), g.dx, LAM,
                                  N0, z_f))
    ref = amp * np.exp(1j * phi.astype(float)) * np.exp(-1j * kz * z_f)
    assert np.abs(spec - ref).max() <= 1e-6
    rng = np.random.default_rng(2)
    G = (rng.standard_normal(spec.shape) + 1j * rng.standard_normal(spec.shape)).astype(np.complex64)
    gp = cpu(bpm.pupil_phase_grad(to_gpu(G, np.complex64), to_gpu(spec, np.complex64)))
    assert np.abs(gp - np.imag(G * np.conj(spec))).max() <= 1e-5


def batch_case(nx, ny, steps, seed):
    """Jobs of one geometry with different gradient requests: the full
    adjoint, a field-only loss with dn gradients, an intensity-only loss, and
    a linear job (no forward field)."""
    rng = np.random.default_rng(seed)
    jobs = []
    for k in range(4):
        u0, w, gI, dn = rand_case(nx, ny, steps, seed=seed * 10 + k)
        jobs.append(dict(field=u0, dn=dn, grad_field_out=w if k != 2 else None,
                         grad_intensity=gI if k in (0, 2) else None,
                         want_spectrum=True, want_dn=k != 3))
    jobs[3]["field"] = None
    rng.shuffle(jobs)
    return jobs


def gpu_jobs(jobs):
    out = []
    for j in jobs:
        g = dict(j)
        g["dn"] = to_gpu(j["dn"], np.float32)
        for key in ("field", "grad_field_out"):
            if j.get(key) is not None:
                g[key] = to_gpu(j[key], np.complex64)
        if j.get("grad_intensity") is not None:
            g["grad_intensity"] = to_gpu(j["grad_intensity"], np.float32)
        out.append(g)
    return out


def separate(jobs, ck=0):
    import paper_1706_02261_amd as bpm
    res = []
    for j in jobs:
        res.append(bpm.adjoint(j.get("field"), j["dn"], 0.2, 0.2, LAM, N0,
                               grad_field_out=j.get("grad_field_out"),
                               grad_intensity=j.get("grad_intensity"),
                               want_spectrum=j.get("want_spectrum", False),
                               want_dn=j.get("want_dn", True), checkpoint_every=ck))
    torch.cuda.synchronize()
    return res


def same(a, b):
    return (a is None and b is None) or torch.equal(a, b)


@pytest.mark.parametrize("nx,ny,steps,n,ck", [(256, 256, 40, 4, 0), (64, 128, 9, 3, 2),
                                              (1024, 64, 6, 2, 0), (128, 128, 1, 4, 1),
                                              (256, 256, 12, 8, 5)])
def test_adjoint_batch_equals_separate_calls(nx, ny, steps, n, ck):
    """Lockstep adjoints of several fields give the bits of separate calls,
    for mixed gradient requests (full, field-only, intensity-only, linear)."""
    import paper_1706_02261_amd as bpm
    cases = batch_case(nx, ny, steps, seed=nx + steps + n)
    jobs = gpu_jobs([cases[k % 4] for k in range(n)])
    got = bpm.adjoint_batch(jobs, 0.2, 0.2, LAM, N0, checkpoint_every=ck)
    torch.cuda.synchronize()
    ref = separate(jobs, ck)
    for k, (g, r) in enumerate(zip(got, ref)):
        assert all(same(a, b) for a, b in zip(g, r)), k


def test_adjoint_batch_linear_jobs_match_oracle():
    """A batch of linear jobs only (no forward field, no dn gradient) takes
    the linear path; each job agrees with the oracle's M^H and with its
    separate call bit for bit."""
    import paper_1706_02261_amd as bpm
    nx, ny, steps = 128, 64, 12
    jobs, cases = [], []
    for k in range(3):
        u0, w, gI, dn = rand_case(nx, ny, steps, seed=70 + k)
        cases.append((u0, w, dn))
        jobs.append(dict(dn=to_gpu(dn, np.float32), grad_field_out=to_gpu(w, np.complex64),
                         want_dn=False, want_spectrum=True))
    got = bpm.adjoint_batch(jobs, 0.2, 0.2, LAM, N0)
    torch.cuda.synchronize()
    ref = separate(jobs)
    for k, ((g0, gs, gdn), (r0, rs, rdn)) in enumerate(zip(got, ref)):
        assert gdn is None and torch.equal(g0, r0) and torch.equal(gs, rs)
        u0, w, dn = cases[k]
        o0, os_, _ = oracle.bpm_adjoint(u0, dn, 0.2, 0.2, LAM, N0, grad_u_out=w,
                                        grad_intensity=None)
        assert rel(cpu(g0), o0) <= 2e-5 and rel(cpu(gs), os_) <= 2e-5


def test_adjoint_batch_zero_steps():
    """Zero steps: g_0 = dL/du_N for every job (and its spectrum)."""
    import paper_1706_02261_amd as bpm
    rng = np.random.default_rng(5)
    ws = [(rng.standard_normal((32, 64)) + 1j * rng.standard_normal((32, 64))).astype(np.complex64)
          for _ in range(2)]
    jobs = [dict(field=to_gpu(w, np.complex64), dn=torch.zeros((0, 32, 64), device="cuda"),
                 grad_field_out=to_gpu(w, np.complex64), want_spectrum=True) for w in ws]
    got = bpm.adjoint_batch(jobs, 0.2, 0.2, LAM, N0)
    torch.cuda.synchronize()
    for (g0, gs, gdn), w in zip(got, ws):
        assert np.array_equal(cpu(g0), w)
        assert rel(cpu(gs), np.fft.fft2(w) / w.size) <= 1e-6
        assert gdn.shape == (0, 32, 64)
