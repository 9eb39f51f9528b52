"""GPU parity at the workloads' full sizes and on the 2048-wide layouts.

* the 512^2 x 512 multiplexed-PSF workload (256 sources, sphere + noise
  phantom), field and whole intensity volume against the FP64 oracle;
* the paper-scale 1024^2 x 1024 detection march, alone (bpm_propagate) and
  in the two-field lockstep launch with the light-sheet march that the
  benchmark times (bpm_propagate_batch), both fields and both intensity
  volumes against the oracle;
* rows of 2048 (two wavefronts per row) where a workgroup transforms several
  row units back to back: a 2048 x 1024 and a 2048^2 march, a 2048-wide job
  in the work-queue batch, and a 2048 x 512 adjoint whose passes mix adjoint
  and recompute units.

Tolerance: relative L2 <= 1e-3 for the runs of 512 and 1024 steps (FP32 FFT
error ~1e-7 log2 N per pass, accumulated over ~sqrt(steps) passes, stays two
orders below); short runs <= 2e-6 (field) and 4e-6 (intensity) as in the
size sweep.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def random_case(nx, ny, steps, seed):
    rng = np.random.default_rng(seed)
    u0 = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
    dn = rng.uniform(0, 0.05, (steps, ny, nx)).astype(np.float32)
    return u0, dn


def gpu_march(u0, dn, g):
    import paper_1706_02261_amd as bpm
    out, inten = bpm.propagate(torch.from_numpy(u0).cuda(), torch.from_numpy(dn).cuda(), g.dx,
                               g.dz, g.wavelength, g.n0)
    torch.cuda.synchronize()
    return out.cpu().numpy(), inten.cpu().numpy()


@pytest.mark.timeout(600)
def test_multiplexed_psf_workload_full_size():
    """512^2 x 512, 256 multiplexed sources: field and intensity volume <= 1e-3."""
    g, u0, dn = synth.config1()
    print("512^2 x 512 workload generated", flush=True)
    u, inten = gpu_march(u0, dn, g)
    ru, ri = oracle.bpm_forward(u0, dn, g.dx, g.dz, g.wavelength, g.n0)
    eu, ei = rel(u, ru), rel(inten, ri)
    print(f"512^2 x 512: field {eu:.3e} intensity {ei:.3e}", flush=True)
    assert eu <= 1e-3 and ei <= 1e-3


@pytest.fixture(scope="module")
def paper_scale():
    """The paper-scale workload and its FP64 oracle results (float32 copies
    of the intensity volumes, to bound host memory)."""
    g, u0, dn = synth.config2_detection()
    gl, u0_ls, dn_ls = synth.config2_light_sheet(g, dn)
    print("paper-scale inputs generated", flush=True)
    ref = []
    for uu, dd in ((u0, dn), (u0_ls, dn_ls)):
        ru, ri = oracle.bpm_forward(uu, dd, g.dx, g.dz, g.wavelength, g.n0)
        ref.append((ru, ri.astype(np.float32)))
        del ri
        print("oracle march done", flush=True)
    return dict(g=g, inputs=[(u0, dn), (u0_ls, dn_ls)], ref=ref)


@pytest.mark.timeout(900)
def test_paper_scale_detection_march(paper_scale):
    """1024^2 x 1024 detection field alone (the single-field kernel)."""
    g = paper_scale["g"]
    u0, dn = paper_scale["inputs"][0]
    u, inten = gpu_march(u0, dn, g)
    ru, ri = paper_scale["ref"][0]
    eu, ei = rel(u, ru), rel(inten, ri)
    print(f"1024^3 detection: field {eu:.3e} intensity {ei:.3e}", flush=True)
    assert eu <= 1e-3 and ei <= 1e-3


@pytest.mark.timeout(900)
def test_paper_scale_lockstep_launch(paper_scale):
    """Detection and light-sheet marches in the two-field lockstep launch that
    the benchmark times."""
    import paper_1706_02261_amd as bpm
    g = paper_scale["g"]
    jobs = [dict(field=torch.from_numpy(uu).cuda(), dn=torch.from_numpy(dd).cuda(), dx=g.dx,
                 dz=g.dz, wavelength=g.wavelength, n0=g.n0)
            for uu, dd in paper_scale["inputs"]]
    res = bpm.propagate_batch(jobs)
    torch.cuda.synchronize()
    del jobs
    for name, (o, i), (ru, ri) in zip(("detection", "light sheet"), res, paper_scale["ref"]):
        eu = rel(o.cpu().numpy(), ru)
        ei = rel(i.cpu().numpy(), ri)
        print(f"1024^3 lockstep {name}: field {eu:.3e} intensity {ei:.3e}", flush=True)
        assert eu <= 1e-3 and ei <= 1e-3


@pytest.mark.parametrize("nx,ny,steps", [(2048, 1024, 3), (2048, 2048, 2)])
def test_2048_wide_rows_several_units_per_workgroup(nx, ny, steps):
    """More row units than workgroups: the head and tail passes run several
    natural-order row units back to back in one workgroup."""
    u0, dn = random_case(nx, ny, steps, seed=nx + ny)
    g = synth.Geometry(nx, ny, steps, 0.2, 0.2)
    u, inten = gpu_march(u0, dn, g)
    ru, ri = oracle.bpm_forward(u0, dn, g.dx, g.dz, g.wavelength, g.n0)
    assert rel(u, ru) <= 2e-6 and rel(inten, ri) <= 4e-6


def test_2048_wide_job_in_the_work_queue_batch():
    import paper_1706_02261_amd as bpm
    shapes = [(2048, 256, 3), (256, 256, 5), (2048, 64, 2)]
    jobs = []
    for i, (nx, ny, st) in enumerate(shapes):
        u0, dn = random_case(nx, ny, st, seed=40 + i)
        jobs.append(dict(u0=u0, dn_h=dn, field=torch.from_numpy(u0).cuda(),
                         dn=torch.from_numpy(dn).cuda(), dx=0.2, dz=0.2, wavelength=0.5,
                         n0=1.33))
    res = bpm.propagate_batch(jobs)
    torch.cuda.synchronize()
    for j, (o, i) in zip(jobs, res):
        so, si = bpm.propagate(j["field"], j["dn"], 0.2, 0.2, 0.5, 1.33)
        assert torch.equal(o, so) and torch.equal(i, si)
        ru, ri = oracle.bpm_forward(j["u0"], j["dn_h"], 0.2, 0.2, 0.5, 1.33)
        assert rel(o.cpu().numpy(), ru) <= 2e-6 and rel(i.cpu().numpy(), ri) <= 4e-6


def test_2048_wide_adjoint_with_mixed_passes():
    """2048 x 512, 5 steps, checkpoints every 2: the passes that carry an
    adjoint step and a recompute step hold two row units per workgroup."""
    import paper_1706_02261_amd as bpm
    nx, ny, steps = 2048, 512, 5
    rng = np.random.default_rng(77)
    u0, dn = random_case(nx, ny, steps, seed=78)
    w = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
    gI = rng.standard_normal((steps, ny, nx)).astype(np.float32)
    g0, gs, gdn = bpm.adjoint(torch.from_numpy(u0).cuda(), torch.from_numpy(dn).cuda(), 0.2, 0.2,
                              0.5, 1.33, grad_field_out=torch.from_numpy(w).cuda(),
                              grad_intensity=torch.from_numpy(gI).cuda(), want_spectrum=True,
                              checkpoint_every=2)
    torch.cuda.synchronize()
    r0, rs, rdn = oracle.bpm_adjoint(u0, dn, 0.2, 0.2, 0.5, 1.33, grad_u_out=w, grad_intensity=gI)
    e = [rel(g0.cpu().numpy(), r0), rel(gs.cpu().numpy(), rs), rel(gdn.cpu().numpy(), rdn)]
    print(f"2048 x 512 adjoint: g0 {e[0]:.2e} spectrum {e[1]:.2e} dn {e[2]:.2e}", flush=True)
    assert max(e) <= 2e-5         # the tolerance of the adjoint size sweep
