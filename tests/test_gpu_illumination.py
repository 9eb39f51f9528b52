"""GPU marches of the alternative light-sheet illuminations (Bessel beam,
bound hexagonal Bessel lattice) through a Perlin-noise tissue, against the
FP64 oracle (field and every intensity slice)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("kind", ["bessel", "lattice"])
def test_illumination_march(kind):
    import paper_1706_02261_amd as bpm
    g = synth.Geometry(256, 256, 48, 0.2, 0.2, 0.5, 1.33)
    dn = synth.perlin_phantom(g, sigma=0.01, gen=synth.rng(6, 1))
    if kind == "bessel":
        u0 = synth.bessel_field(g.nx, g.ny, g.dx, g.wavelength, g.n0, 0.55, 0.45)
    else:
        u0 = synth.bessel_lattice_field(g.nx, g.ny, g.dx, g.wavelength, g.n0, 0.55, 0.45, 6,
                                        (0.08, 0.01))
    out, inten = bpm.propagate(torch.from_numpy(u0).cuda(), torch.from_numpy(dn).cuda(), g.dx,
                               g.dz, g.wavelength, g.n0, intensity=True)
    r_out, r_int = oracle.bpm_forward(u0, dn, g.dx, g.dz, g.wavelength, g.n0)
    assert rel(out.cpu().numpy(), r_out) <= 2e-5
    assert rel(inten.cpu().numpy(), r_int) <= 2e-5
