"""The launch-shape tuner: every eligible kernel of a shape gives the same
bits, the tuner records a choice per shape and its JSON cache re-applies it
in the same process after the choices were cleared."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def jobs_of(nx, ny, fields, steps, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    return [dict(field=torch.randn((ny, nx), dtype=torch.complex64, device="cuda", generator=g),
                 dn=torch.rand((steps, ny, nx), device="cuda", generator=g) * 0.05,
                 dx=0.2, dz=0.2, wavelength=0.5, n0=1.33) for _ in range(fields)]


@pytest.mark.parametrize("shape", [(1024, 1024, 2), (512, 512, 3), (2048, 512, 2), (256, 128, 1),
                                   (128, 128, 1), (32, 1024, 1), (1024, 32, 2), (64, 64, 5),
                                   (1024, 1024, 1)])
def test_every_kernel_of_a_shape_gives_the_same_bits(shape):
    import paper_1706_02261_amd as bpm
    from paper_1706_02261_amd import tune
    nx, ny, fields = shape
    jobs = jobs_of(nx, ny, fields, 5, seed=nx + fields)
    variants = tune.eligible(nx, ny, fields)
    assert tune.VARIANTS and variants and 1 in variants
    res = {}
    try:
        for v in variants:
            tune.set_variant(nx, ny, fields, v)
            assert tune.current_variant(nx, ny, fields) == v
            out = bpm.propagate_batch(jobs)
            torch.cuda.synchronize()
            res[v] = [(o.clone(), i.clone()) for o, i in out]
    finally:
        tune.set_variant(nx, ny, fields, 0)
    first = res[variants[0]]
    for v in variants[1:]:
        for (a, ai), (b, bi) in zip(first, res[v]):
            assert torch.equal(a, b) and torch.equal(ai, bi), v


def test_tuner_records_and_reloads_choices(tmp_path):
    from paper_1706_02261_amd import tune
    shapes = [(1024, 1024, 2), (512, 512, 2)]
    try:
        r = tune.tune(shapes, steps=8, reps=3)
        for sh in shapes:
            assert r[sh]["variant"] in tune.eligible(*sh)
            assert len(r[sh]["ms"]) == len(tune.eligible(*sh))
            assert tune.current_variant(*sh) == r[sh]["variant"]
        print(r, flush=True)
        path = tune.save(r, path=str(tmp_path / "v.json"))
        for sh in shapes:
            tune.set_variant(*sh, 0)
        applied = tune.load(path=path)
        assert applied == {sh: r[sh]["variant"] for sh in shapes}
    finally:
        for sh in shapes:
            tune.set_variant(*sh, 0)
