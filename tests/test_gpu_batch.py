"""GPU parity of the uneven batch (bpm_propagate_batch).

Every job of a batch must equal, bit for bit, its own bpm_propagate call
(same kernels, same plan), and therefore the oracle within the march's
tolerance; jobs of every size class, a zero-step job and repeated launches
on the same workspace are covered.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def make_jobs(shapes, seed):
    rng = np.random.default_rng(seed)
    jobs = []
    for (nx, ny, steps) in shapes:
        u0 = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
        dn = rng.uniform(0, 0.05, (steps, ny, nx)).astype(np.float32)
        dx = float(rng.choice([0.1, 0.2]))
        jobs.append(dict(u0=u0, dn_h=dn, field=torch.from_numpy(u0).cuda(),
                         dn=torch.from_numpy(dn).cuda(), dx=dx, dz=0.2, wavelength=0.5, n0=1.33))
    return jobs


def separate(job):
    import paper_1706_02261_amd as bpm
    out, inten = bpm.propagate(job["field"], job["dn"], job["dx"], job["dz"], job["wavelength"],
                               job["n0"])
    return out.cpu().numpy(), inten.cpu().numpy()


SHAPES = [(64, 128, 5), (256, 256, 12), (32, 32, 0), (128, 64, 7), (512, 128, 3),
          (1024, 32, 2), (32, 2048, 4), (256, 512, 9)]


def test_batch_equals_separate_calls_and_oracle():
    import paper_1706_02261_amd as bpm
    jobs = make_jobs(SHAPES, seed=1)
    res = bpm.propagate_batch(jobs)
    torch.cuda.synchronize()
    for job, (out, inten) in zip(jobs, res):
        o, i = out.cpu().numpy(), inten.cpu().numpy()
        so, si = separate(job)
        assert np.array_equal(o, so) and np.array_equal(i, si), job["u0"].shape
        steps = job["dn_h"].shape[0]
        if steps == 0:
            assert np.array_equal(o, job["u0"])
            continue
        ro, ri = oracle.bpm_forward(job["u0"], job["dn_h"], job["dx"], job["dz"], 0.5, 1.33)
        assert rel(o, ro) <= 2e-6 and rel(i, ri) <= 4e-6


# columns of >= 1024 with nx >= 256 and nx ny <= 2^20 stay in the tiled layout
# between the work queue's passes; (128, 1024) and (1024, 256) do not
TILED_SHAPES = [(256, 1024, 5), (512, 1024, 4), (1024, 1024, 3), (256, 2048, 3),
                (512, 2048, 2), (256, 1024, 1), (128, 1024, 3), (1024, 256, 4)]


def test_work_queue_tiled_jobs_equal_separate_calls_and_oracle():
    """Jobs the work queue keeps tiled between passes, one-step jobs among
    them, next to natural-layout jobs: the bits of separate calls, and the
    oracle within the march's tolerance."""
    import paper_1706_02261_amd as bpm
    jobs = make_jobs(TILED_SHAPES, seed=12)
    res = bpm.propagate_batch(jobs)
    torch.cuda.synchronize()
    for job, (out, inten) in zip(jobs, res):
        o, i = out.cpu().numpy(), inten.cpu().numpy()
        so, si = separate(job)
        assert np.array_equal(o, so) and np.array_equal(i, si), job["u0"].shape
        ro, ri = oracle.bpm_forward(job["u0"], job["dn_h"], job["dx"], job["dz"], 0.5, 1.33)
        assert rel(o, ro) <= 2e-6 and rel(i, ri) <= 4e-6, job["u0"].shape


def test_batch_repeated_launches_on_one_workspace():
    """Queue and completion counters are reset by every launch."""
    import paper_1706_02261_amd as bpm
    from paper_1706_02261_amd import _lib
    from paper_1706_02261_amd.bpm import workspace
    jobs = make_jobs([(256, 256, 20), (512, 512, 6), (128, 256, 33)], seed=2)
    first = [(o.clone(), i.clone()) for o, i in bpm.propagate_batch(jobs)]
    torch.cuda.synchronize()
    for _ in range(3):
        again = bpm.propagate_batch(jobs)
        torch.cuda.synchronize()
        for (a, ai), (b, bi) in zip(first, again):
            assert torch.equal(a, b) and torch.equal(ai, bi)


def test_batch_of_the_uneven_mix():
    """16 jobs drawn like the paper-scale batch (sizes 256-1024, random depth),
    each compared bitwise with its own march."""
    import paper_1706_02261_amd as bpm
    specs = synth.batch_job_specs(n_jobs=16, steps_range=(4, 24), budget_bytes=4e9, seed_child=11)
    jobs = make_jobs(specs, seed=3)
    res = bpm.propagate_batch(jobs)
    torch.cuda.synchronize()
    for job, (out, inten) in zip(jobs, res):
        so, si = separate(job)
        assert np.array_equal(out.cpu().numpy(), so) and np.array_equal(inten.cpu().numpy(), si)


@pytest.mark.parametrize("shape,n_jobs", [((256, 512, 9), 3), ((128, 128, 5), 8),
                                          ((64, 64, 3), 9), ((1024, 1024, 6), 2),
                                          ((1024, 1024, 4), 3), ((1024, 1024, 3), 8),
                                          ((2048, 512, 3), 2), ((512, 2048, 3), 4)])
def test_lockstep_batch_of_one_geometry(shape, n_jobs):
    """Jobs of one geometry (up to 8) march in lockstep in the cooperative
    kernel (the pipelined one where every pass of a field has one unit per CU:
    1024^2, 2048 x 512, 512 x 2048); 9 fall back to the work queue.  Either way every job equals its own
    march bit for bit; one job writes its output over its input and one skips
    the intensity volume."""
    import paper_1706_02261_amd as bpm
    jobs = make_jobs([shape] * n_jobs, seed=4 + n_jobs)
    for j in jobs:
        j["dx"] = 0.2
    ref = [separate(j) for j in jobs]
    jobs[0]["out"] = jobs[0]["field"].clone()
    jobs[0]["field"] = jobs[0]["out"]
    jobs[-1]["intensity"] = False
    res = bpm.propagate_batch(jobs)
    torch.cuda.synchronize()
    for k, (job, (out, inten)) in enumerate(zip(jobs, res)):
        assert np.array_equal(out.cpu().numpy(), ref[k][0]), k
        if k == n_jobs - 1:
            assert inten is None
        else:
            assert np.array_equal(inten.cpu().numpy(), ref[k][1]), k


def test_prepared_batch_in_a_captured_graph():
    """The device half of the batch (bpm_batch_launch) captured into a graph:
    three replays, each after new inputs were written into the captured
    tensors, each equal bit for bit to separate marches of those inputs; and a
    launch on a workspace that holds no tables leaves the outputs untouched."""
    import paper_1706_02261_amd as bpm
    from paper_1706_02261_amd import _lib
    from paper_1706_02261_amd.bpm import _ptr, _stream_ptr
    jobs = make_jobs([(64, 128, 5), (256, 256, 7), (32, 32, 0), (128, 64, 4)], seed=21)
    prep = bpm.PreparedBatch(jobs)
    first = [(o.clone(), None if i is None else i.clone()) for o, i in prep.launch()]
    torch.cuda.synchronize()
    for job, (o, i) in zip(jobs, first):
        so, si = separate(job)
        assert np.array_equal(o.cpu().numpy(), so)
        assert i is None or np.array_equal(i.cpu().numpy(), si)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        prep.launch()
    torch.cuda.synchronize()
    gen = np.random.default_rng(6)
    for rep in range(3):
        for job in jobs:
            ny, nx = job["field"].shape
            u = gen.standard_normal((ny, nx)) + 1j * gen.standard_normal((ny, nx))
            job["field"].copy_(torch.from_numpy(u.astype(np.complex64)))
            job["dn"].copy_(torch.from_numpy(
                gen.uniform(0, 0.05, tuple(job["dn"].shape)).astype(np.float32)))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, (job, (o, i)) in enumerate(zip(jobs, prep.results)):
            so, si = separate(job)
            assert np.array_equal(o.cpu().numpy(), so), (rep, k)
            assert i is None or np.array_equal(i.cpu().numpy(), si), (rep, k)
    # a workspace without tables: the batch kernel takes no item
    for o, i in prep.results:
        o.fill_(7.0)
        if i is not None:
            i.fill_(7.0)
    empty = torch.zeros_like(prep.ws)
    rc = _lib.lib().bpm_batch_launch(prep._arr, len(jobs), _ptr(empty), empty.numel(),
                                     _stream_ptr(None))
    torch.cuda.synchronize()
    assert rc == 0
    for job, (o, i) in zip(jobs, prep.results):
        if job["dn"].shape[0] > 0:
            assert bool((o == 7.0).all()) and (i is None or bool((i == 7.0).all()))


def test_captured_graph_of_the_64_job_mix():
    """The 64-job uneven mix (sizes 256-1024 drawn like the paper-scale batch,
    steps cut to 2-6) captured into one graph: two replays, each job equal bit
    for bit to its own march."""
    import paper_1706_02261_amd as bpm
    specs = synth.batch_job_specs(n_jobs=64, steps_range=(2, 6), budget_bytes=8e9,
                                  seed_child=12)
    jobs = make_jobs(specs, seed=64)
    ref = [separate(j) for j in jobs]
    prep = bpm.PreparedBatch(jobs)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        prep.launch()
    for rep in range(2):
        for o, i in prep.results:
            o.fill_(0.0)
            i.fill_(0.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, (o, i) in enumerate(prep.results):
            assert np.array_equal(o.cpu().numpy(), ref[k][0]), (rep, k)
            assert np.array_equal(i.cpu().numpy(), ref[k][1]), (rep, k)


# ---------------------------------------------------------------------------
# staggered starts (clear_steps)

def _clear_case(nx, ny, steps, k, seed):
    rng = np.random.default_rng(seed)
    u = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
    dn = rng.uniform(0, 0.05, (steps, ny, nx)).astype(np.float32)
    zeroed = dn.copy()
    zeroed[:k] = 0.0
    return u, dn, zeroed


@pytest.mark.parametrize("shape", [(256, 256, 9, 2), (1024, 1024, 6, 2), (128, 64, 7, 3),
                                   (512, 512, 5, 1)])
def test_clear_steps_equal_a_zeroed_prefix(shape):
    """Jobs whose first k screens are skipped give the bits of jobs whose
    first k dn slices are zero, in the lockstep kernels and the work queue."""
    import paper_1706_02261_amd as bpm
    nx, ny, steps, fields = shape
    ks = [3, 0, steps][:fields]
    cases = [_clear_case(nx, ny, steps, k, seed=nx + 7 * k) for k in ks]
    def jobs(clear):
        out = []
        for (u, dn, zeroed), k in zip(cases, ks):
            out.append(dict(field=torch.from_numpy(u).cuda(),
                            dn=torch.from_numpy(dn if clear else zeroed).cuda(), dx=0.2, dz=0.2,
                            wavelength=0.5, n0=1.33, clear_steps=k if clear else 0))
        return out
    a = bpm.propagate_batch(jobs(True))
    b = bpm.propagate_batch(jobs(False))
    # the work queue: an extra job of another size forces the uneven path
    extra = dict(field=torch.zeros((32, 32), dtype=torch.complex64, device="cuda"),
                 dn=torch.zeros((2, 32, 32), device="cuda"), dx=0.2, dz=0.2, wavelength=0.5,
                 n0=1.33)
    c = bpm.propagate_batch(jobs(True) + [extra])[:len(ks)]
    torch.cuda.synchronize()
    for (oa, ia), (ob, ib), (oc, ic) in zip(a, b, c):
        assert torch.equal(oa, ob) and torch.equal(ia, ib)
        assert torch.equal(oc, ob) and torch.equal(ic, ib)


def test_staggered_start_matches_the_march_from_depth():
    """A source entered k slices early, defocused by k dz, with k cleared
    steps, leaves the volume as the oracle's in-focus source marched from
    slice k."""
    import paper_1706_02261_amd as bpm
    n, steps, k = 256, 20, 7
    rng = np.random.default_rng(12)
    dn = rng.uniform(0, 0.04, (steps, n, n)).astype(np.float32)
    src = np.array([[40, 50], [200, 130]], np.int32)
    u_early = bpm.point_sources(torch.from_numpy(src).cuda(), n, n, 0.2, 0.5, 1.33, 0.6, k * 0.2)
    (out, _), = bpm.propagate_batch([dict(field=u_early, dn=torch.from_numpy(dn).cuda(), dx=0.2,
                                          dz=0.2, wavelength=0.5, n0=1.33, clear_steps=k,
                                          intensity=False)])
    u0 = oracle.point_sources(n, n, 0.2, 0.5, 1.33, 0.6, 0.0, src)
    ref, _ = oracle.bpm_forward(u0, dn[k:], 0.2, 0.2, 0.5, 1.33, intensity=False)
    got = out.cpu().numpy()
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 2e-5
