"""The synthetic workloads and the benchmark's reference figure against the
numbers the paper prints (tests/golden/paper_parameters.json)."""
import json
import os

import numpy as np

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
P = {k: v["value"] for k, v in json.load(open(os.path.join(HERE, "golden",
                                                           "paper_parameters.json"))).items()
     if not k.startswith("_")}
N0 = 1.33


def test_phantom_index_ranges():
    g, _, dn = synth.config2_detection(steps=32, nxy=128)
    lo, hi = P["tissue_phantom_n_range"]
    assert g.n0 == lo
    assert N0 + dn.min() >= lo - 1e-7 and N0 + dn.max() <= hi + 1e-7
    _, dn3, _, _ = synth.config3(steps=16, nxy=64)
    assert N0 + dn3.max() <= P["embryo_model_n_range"][1] + 1e-7
    v = synth.surrogate_volume(0, nxy=64, nz=64)
    assert N0 + v.min() >= lo - 1e-7 and N0 + v.max() <= hi + 1e-7


def test_paper_scale_geometry_holds_the_phantom():
    # dx = dz = 0.2 um: the 1024^3 grid spans 204.8 um, enough for 100 x 200 x 100 um
    extent = 1024 * 0.2
    assert max(P["tissue_phantom_size_um"]) <= extent
    assert tuple(P["march_volume_voxels"]) == (1024, 1024, 1024)


def test_source_and_sheet_apertures():
    # the generators put no power outside the printed apertures
    nx = 128
    spec = synth.point_source_spectrum(nx, nx, 0.2, 0.5, N0, P["detection_na"], 0.0)
    f = 2 * np.pi * np.fft.fftfreq(nx, d=0.2)
    kt = np.sqrt(f[None, :] ** 2 + f[:, None] ** 2)
    k0 = 2 * np.pi / 0.5
    assert np.abs(spec[kt > k0 * P["detection_na"] + 1e-9]).max() == 0.0
    sheet = synth.light_sheet_field(nx, nx, 0.2, 0.5, N0, P["illumination_na"], 5.0)
    S = np.fft.fft2(sheet)
    assert np.abs(S[kt > k0 * P["illumination_na"] + 1e-9]).max() <= 1e-6 * np.abs(S).max()


def test_benchmark_reference_figure():
    import bench
    ref = np.prod(P["march_volume_voxels"]) / P["march_time_upper_s"] / 1e9
    assert abs(bench.PAPER_GVS - ref) <= 1e-12
