"""A wait that gives up inside a persistent kernel is reported by the
workspace's status query (bpm_workspace_status), not silently as success.

The time-out is forced from the host: the process-wide wait bound is set to a
single poll, so the first grid-barrier (or queue) wait of each workgroup that
is not released at once gives up; the kernel then stops waiting and runs to
its end (every access of the march is data-independent and in bounds, so its
outputs are merely wrong).  With the default bound restored, the next call on
the same workspace is correct again and the query reports success.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def case(nx, ny, steps, seed):
    rng = np.random.default_rng(seed)
    u0 = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
    dn = rng.uniform(0, 0.05, (steps, ny, nx)).astype(np.float32)
    return u0, dn


@pytest.fixture
def restore_limit():
    import paper_1706_02261_amd as bpm
    yield
    bpm.set_wait_limit(0)


def test_fresh_workspace_has_no_status():
    import paper_1706_02261_amd as bpm
    from paper_1706_02261_amd import _lib
    ws = torch.zeros(bpm.workspace_size(64, 64, 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(_lib.BpmError) as e:
        bpm.workspace_status(ws)
    assert e.value.code == _lib.BPM_ERR_INVALID_ARG


def test_march_time_out_is_reported(restore_limit):
    import paper_1706_02261_amd as bpm
    from paper_1706_02261_amd import _lib
    u0, dn = case(512, 512, 16, 1)
    f, d = torch.from_numpy(u0).cuda(), torch.from_numpy(dn).cuda()
    ws = bpm.workspace(bpm.workspace_size(512, 512, 16), f.device)
    print("march with a one-poll wait bound", flush=True)
    bpm.set_wait_limit(1)
    bpm.propagate(f, d, 0.2, 0.2, 0.5, 1.33, ws=ws)
    with pytest.raises(_lib.BpmError) as e:
        bpm.workspace_status(ws)
    assert e.value.code == _lib.BPM_ERR_DEVICE and "grid-barrier" in str(e.value)
    bpm.workspace_status(ws)          # the query reset the record
    bpm.set_wait_limit(0)
    out, inten = bpm.propagate(f, d, 0.2, 0.2, 0.5, 1.33, ws=ws)
    bpm.workspace_status(ws)
    fresh, fresh_i = bpm.propagate(f, d, 0.2, 0.2, 0.5, 1.33)     # a workspace never timed out
    assert torch.equal(out, fresh) and torch.equal(inten, fresh_i)
    ru, ri = oracle.bpm_forward(u0, dn, 0.2, 0.2, 0.5, 1.33)
    assert rel(out.cpu().numpy(), ru) <= 1e-5 and rel(inten.cpu().numpy(), ri) <= 1e-5


def test_batch_queue_time_out_is_reported(restore_limit):
    import paper_1706_02261_amd as bpm
    from paper_1706_02261_amd import _lib
    shapes = [(256, 256, 6), (128, 512, 5), (512, 128, 4)]
    jobs = []
    for i, (nx, ny, st) in enumerate(shapes):
        u0, dn = case(nx, ny, st, 10 + i)
        jobs.append(dict(u0=u0, dn_h=dn, field=torch.from_numpy(u0).cuda(),
                         dn=torch.from_numpy(dn).cuda(), dx=0.2, dz=0.2, wavelength=0.5,
                         n0=1.33))
    from paper_1706_02261_amd import bpm as B
    ws = bpm.workspace(B._batch_table(jobs)[2], "cuda")
    print("uneven batch with a one-poll wait bound", flush=True)
    bpm.set_wait_limit(1)
    bpm.propagate_batch(jobs, ws=ws)
    with pytest.raises(_lib.BpmError) as e:
        bpm.workspace_status(ws)
    assert e.value.code == _lib.BPM_ERR_DEVICE and "work-queue" in str(e.value)
    bpm.set_wait_limit(0)
    res = bpm.propagate_batch(jobs, ws=ws)
    bpm.workspace_status(ws)
    for j, (o, i) in zip(jobs, res):
        so, si = bpm.propagate(j["field"], j["dn"], 0.2, 0.2, 0.5, 1.33)
        assert torch.equal(o, so) and torch.equal(i, si)
        ru, ri = oracle.bpm_forward(j["u0"], j["dn_h"], 0.2, 0.2, 0.5, 1.33)
        assert rel(o.cpu().numpy(), ru) <= 1e-5 and rel(i.cpu().numpy(), ri) <= 1e-5
