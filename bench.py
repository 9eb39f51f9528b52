#!/usr/bin/env python3
"""Benchmark of the split-step beam-propagation march on one MI355X.

Timed step: the paper-scale workload -- the detection march (a 1024 x 1024
complex64 field carrying 1000 multiplexed NA 0.6 point sources through 1024
slices of an embryo-like ellipsoid phantom, dx = dz = 0.2 um, lambda = 0.5 um,
n0 = 1.33) and the light-sheet march (NA 0.15 sheet through the same volume
along the orthogonal axis), both intensity volumes written, in one lockstep
launch through the C ABI (bpm_propagate_batch), inputs resident in HBM.
Prints ONE JSON line:

  value      Gvoxel-steps/s = fields * nx * ny * slices / t_step
  roofline   HBM model: 40 bytes per voxel-step (two read+write passes over
             the complex64 field, the dn slice read, the intensity write)
             against 8 TB/s; `traffic` is the memory traffic rocprofv3 measured
             for one launch (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known
             size) divided by this run's launch time, in GB/s, when the
             committed counter summary matches the current kernel source, else
             null
  psf        surrogate vs BPM PSFs/s on the PSF volumes of the surrogate
  cpu_baseline  the FP64 oracle on the machine's host cores over a bounded sample
             (the first slices of the same volume), with the relative L2
             error of the GPU field against it on that sample

`--gpus N` with N > 1 exits: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BPM Gvoxel-steps/s at 1024³ c64 (% HBM roofline); surrogate vs BPM PSFs/s"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
BYTES_PER_VOXEL_STEP = 40
FLOP_PER_VOXEL_STEP = 215          # 10 log2(nx ny) + 15 at 1024^2 (5 N log2 N FFT count)
PAPER_GVS = 1024 ** 3 / 0.5 / 1e9  # < 500 ms for 1024^3 voxels, main text
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "march_1024cube_traffic.json")


MARCH_SOURCES = ("fft.hpp", "mathx.hpp", "passes.hpp", "tiled.hpp", "march_kernels.hpp",
                 "march_x1024.hip", "march.hip")


def kernel_source_hash() -> str:
    """Hash of the sources the march kernel is compiled from."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1706_02261_amd", "csrc")
    for name in MARCH_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 summary, if it was
    taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_gvs(u0, dn, g, reps=1):
    """Median Gvoxel-steps/s of the oracle march (intensity volume included)
    over `reps` runs after one warm-up when reps > 1; seconds of one run."""
    import numpy as np
    import oracle
    ts = []
    for _ in range(reps + (1 if reps > 1 else 0)):
        t0 = time.perf_counter()
        oracle.bpm_forward(u0, dn, g.dx, g.dz, g.wavelength, g.n0)
        ts.append(time.perf_counter() - t0)
    t = float(np.median(ts[1:] if reps > 1 else ts))
    return g.nx * g.ny * dn.shape[0] / t / 1e9, t


def cpu_baseline(u0, dn_host, g, gpu_fn, small, target_s=12.0):
    """The FP64 oracle on the host cores: the paper-scale volume's first slices
    (the bounded sample of the timed workload, with the GPU's error on it),
    the same on one thread, and the 128^2 x 64 and 512^2 x 512 workloads in
    full (the latter on one thread over its first 32 slices)."""
    import numpy as np
    import oracle
    threads = oracle.set_threads(0)
    # per-step time from the second and third steps (the first pays the
    # plan and the first-touch page faults)
    t0 = time.perf_counter()
    oracle.bpm_forward(u0, dn_host[:1], g.dx, g.dz, g.wavelength, g.n0, intensity=False)
    t1 = time.perf_counter()
    oracle.bpm_forward(u0, dn_host[:3], g.dx, g.dz, g.wavelength, g.n0, intensity=False)
    per_step = max((time.perf_counter() - t1) - (t1 - t0), 1e-6) / 2
    steps = int(max(4, min(dn_host.shape[0], target_s / max(per_step, 1e-6))))
    t0 = time.perf_counter()
    ref, _ = oracle.bpm_forward(u0, dn_host[:steps], g.dx, g.dz, g.wavelength, g.n0,
                                intensity=False)
    t = time.perf_counter() - t0
    got = gpu_fn(steps)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    workloads = {}
    for name, (gs, us, ds), reps in ((k, v, 3 if k.startswith("128") else 1)
                                     for k, v in small.items()):
        gvs_n, t_n = _oracle_gvs(us, ds, gs, reps)
        workloads[name] = {"gvoxel_steps_per_s": round(gvs_n, 4), "seconds": round(t_n, 3),
                           "threads": threads}
    try:
        oracle.set_threads(1)
        one = {}
        one_steps = 4
        t0 = time.perf_counter()
        oracle.bpm_forward(u0, dn_host[:one_steps], g.dx, g.dz, g.wavelength, g.n0,
                           intensity=False)
        one["paper_scale_first_4_slices"] = round(g.nx * g.ny * one_steps /
                                                  (time.perf_counter() - t0) / 1e9, 5)
        for name, (gs, us, ds), in small.items():
            cut = ds if name.startswith("128") else ds[:32]
            gvs_1, _ = _oracle_gvs(us, cut, gs, 3 if name.startswith("128") else 1)
            one[name if cut is ds else f"{name}_first_32_slices"] = round(gvs_1, 5)
    finally:
        oracle.set_threads(threads)
    return {"value": round(g.nx * g.ny * steps / t / 1e9, 4), "unit": "Gvoxel-steps/s",
            "cores": threads, "kind": "oracle",
            "sample": f"{g.nx}x{g.ny} field, first {steps} of {g.steps} slices of the timed "
                      f"volume, FP64 radix-2 oracle, OpenMP {threads} threads, "
                      f"{t:.1f} s",
            "cpu_model": cpu_model(), "logical_cpus": os.cpu_count(),
            "one_thread_gvoxel_steps_per_s": one, "workloads": workloads,
            "gpu_rel_l2_err_on_sample": err}


def workload_rates(dev, small, reps=10):
    """The GPU march on the 128^2 x 64 (latency) and 512^2 x 512 workloads
    (bpm_propagate, intensity volume written), median of `reps` launches."""
    import numpy as np
    import torch
    import paper_1706_02261_amd as bpm
    stream = torch.cuda.current_stream(dev)
    out = {}
    for name, (g, u0, dn) in small.items():
        f = torch.from_numpy(u0).to(dev)
        d = torch.from_numpy(dn).to(dev)
        o = torch.empty_like(f)
        inten = torch.empty(dn.shape, dtype=torch.float32, device=dev)
        ws = bpm.workspace(bpm.workspace_size(g.nx, g.ny, g.steps), dev)

        def run():
            bpm.propagate(f, d, g.dx, g.dz, g.wavelength, g.n0, out=o, intensity_out=inten,
                          ws=ws, stream=stream)

        for _ in range(2):
            run()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            run()
            b.record(stream)
            torch.cuda.synchronize(dev)
            ts.append(a.elapsed_time(b))
        ms = float(np.median(ts))
        vs = g.nx * g.ny * g.steps
        gbs = BYTES_PER_VOXEL_STEP * vs / (ms / 1e3) / 1e9
        out[name] = {"ms": round(ms, 4), "gvoxel_steps_per_s": round(vs / (ms / 1e3) / 1e9, 3),
                     "hbm_frac_40B": round(gbs / HBM_PEAK_GBS, 4)}
    return out


SURROGATE_FLOP_PER_PSF = 2 * (8192 * 32 * 27 * 5 + 4096 * 32 * 27 * 32 + 2048 * 32 * 27 * 32
                              + 1024 * 32 * 27 * 32 + 256 * 64 * 36 * 32 + 1024 * 32 * 9 * 64)
MFMA_BF16_PEAK_TFLOPS = 2500.0


def psf_rates(dev, n_runs=8, n_infer=100000, train_seconds=60.0):
    """The learned PSF surrogate against the BPM on the same GPU.

    * BPM PSFs/s: multiplexed runs (1024 sources each, depths spread over the
      64-slice volume; point sources + march + readout);
    * the surrogate is trained for `train_seconds` on 10^5 BPM PSFs of four
      volumes (98 runs) and evaluated on 2048 held-out PSFs of a third:
      relative L2 error against the BPM, the error of the spatially invariant
      clear-medium PSF, the fraction above the 5 % fallback threshold;
    * surrogate PSFs/s on `n_infer` random sources of a fourth volume (patch
      extraction + network + error head), and the effective rate of the whole
      path with the BPM fallback for every source predicted above 5 %."""
    import numpy as np
    import torch
    import synth
    from paper_1706_02261_amd import psfs
    from paper_1706_02261_amd import surrogate as S
    stream = torch.cuda.current_stream(dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    scale = 1.0 / psfs.reference_peak(1024, 1024, device=dev)
    gen = np.random.default_rng(45)

    def runs(vol, n):
        out = [psfs.training_run(vol, int(gen.integers(0, 64)),
                                 (int(gen.integers(0, 32)), int(gen.integers(0, 32))), 32, scale)
               for _ in range(n)]
        return [torch.cat([o[k] for o in out]) for k in range(3)]

    # the training set: 10^5 BPM PSFs (98 multiplexed runs of 1024 sources
    # over four volumes), as the learned part's workload states
    t_gen = time.perf_counter()
    train = [runs(torch.from_numpy(synth.surrogate_volume(c)).to(dev), n)
             for c, n in ((0, 25), (1, 25), (4, 24), (5, 24))]
    X, D, T = (torch.cat([t[k] for t in train]) for k in range(3))
    del train
    torch.cuda.synchronize(dev)
    t_gen = time.perf_counter() - t_gen
    Xv, Dv, Tv = runs(torch.from_numpy(synth.surrogate_volume(2)).to(dev), 2)
    n_train = int(X.shape[0])
    model = S.PSFSurrogate(dev, S.init_params(seed=0))
    epochs = model.fit(X, D, T, seconds=train_seconds)
    del X, D, T
    blob = model.export()
    pred, err = S.infer(blob, Xv, Dv)
    rel = lambda a, b: (a - b).flatten(1).norm(dim=1) / b.flatten(1).norm(dim=1)
    r_s = rel(pred, Tv)
    clear = psfs.bpm_psfs(torch.zeros((64, 1024, 1024), device=dev), 32,
                          torch.tensor([[512, 512]], dtype=torch.int32, device=dev), scale)
    r_inv = rel(clear.expand_as(Tv), Tv)
    q = lambda v, p: round(float(torch.quantile(v.float().cpu(), p)), 4)
    corr = float(np.corrcoef(err.cpu().numpy(), r_s.cpu().numpy())[0, 1])
    # of the held-out PSFs the error head accepts (predicted <= 5 %), the share
    # whose true error against the BPM exceeds 5 %
    acc = err <= 0.05
    accepted_bad = (round(float((r_s[acc] > 0.05).float().mean()), 4) if bool(acc.any())
                    else None)
    del Xv, Dv, Tv, pred

    vol = torch.from_numpy(synth.surrogate_volume(3)).to(dev)
    depths = [int(d) for d in np.linspace(2, 62, n_runs)]

    def bpm_all():
        n = 0
        for i, d in enumerate(depths):
            _, _, t = psfs.training_run(vol, d, (i, 2 * i), 32, scale)
            n += t.shape[0]
        return n

    bpm_all()
    a, b = ev(), ev()
    torch.cuda.synchronize(dev)
    a.record(stream)
    n_bpm = bpm_all()
    b.record(stream)
    torch.cuda.synchronize(dev)
    t_bpm = a.elapsed_time(b) / 1e3
    src = torch.from_numpy(np.stack([gen.integers(0, 64, n_infer), gen.integers(0, 1024, n_infer),
                                     gen.integers(0, 1024, n_infer)], 1).astype(np.int32)).to(dev)

    def timed(threshold):
        a, b = ev(), ev()
        torch.cuda.synchronize(dev)
        a.record(stream)
        _, e, fb = psfs.psf_with_fallback(blob, vol, src, scale, threshold=threshold)
        b.record(stream)
        torch.cuda.synchronize(dev)
        return a.elapsed_time(b) / 1e3, float(fb.float().mean())

    timed(float("inf"))
    t_s, _ = timed(float("inf"))
    t_eff, fb_rate = timed(0.05)
    tflops = SURROGATE_FLOP_PER_PSF * n_infer / t_s / 1e12
    return {
        "bpm_psfs_per_s": round(n_bpm / t_bpm, 1),
        "bpm_sample": f"{n_runs} multiplexed runs of 1024 sources, 1024^2 x (64 - d) slices, "
                      f"d in {depths[0]}..{depths[-1]}, 32-plane readout, 32^3 crops",
        "surrogate_psfs_per_s": round(n_infer / t_s, 1),
        "surrogate_sample": f"{n_infer} random sources (depth, y, x) of a 64 x 1024^2 volume: "
                            "patch extraction + BF16 inference with error head",
        "surrogate_vs_bpm": round((n_infer / t_s) / (n_bpm / t_bpm), 4),
        "effective_psfs_per_s": round(n_infer / t_eff, 1),
        "fallback_rate": round(fb_rate, 4),
        "training": {"psfs": n_train, "seconds": train_seconds, "epochs": epochs,
                     "set_generation_s": round(t_gen, 1)},
        "heldout": {"psfs": 2048, "rel_err_median": q(r_s, 0.5), "rel_err_p95": q(r_s, 0.95),
                    "invariant_psf_rel_err_median": q(r_inv, 0.5),
                    "invariant_psf_rel_err_p95": q(r_inv, 0.95),
                    "error_head_corr": round(corr, 3),
                    "above_5pct": round(float((err > 0.05).float().mean()), 4),
                    "accepted_true_above_5pct": accepted_bad},
        "surrogate_roofline": {"bound": "mfma", "achieved": round(tflops, 2),
                               "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": round(tflops / MFMA_BF16_PEAK_TFLOPS, 5),
                               "flop_per_psf": SURROGATE_FLOP_PER_PSF},
    }


ADJOINT_BYTES_PER_VOXEL_STEP = 128   # checkpoint march + segment recompute + adjoint, whole call


def adjoint_rate(dev, reps=3):
    """The adjoint workload: 256^2 x 512 sphere phantom, gradients of the
    negative focal-spot intensity with respect to the pupil spectrum and dn
    (sqrt(N) checkpoints), one bpm_adjoint call."""
    import numpy as np
    import torch
    import synth
    import paper_1706_02261_amd as bpm
    g, dn_h, amp, z_f = synth.config3()
    dn = torch.from_numpy(dn_h).to(dev)
    phase = torch.zeros((g.ny, g.nx), dtype=torch.float32, device=dev)
    U0 = bpm.pupil_spectrum(torch.from_numpy(amp.astype(np.float32)).to(dev), phase, g.dx,
                            g.wavelength, g.n0, z_f)
    u0 = bpm.fft2(U0, inverse=True)
    gI = torch.zeros((g.steps, g.ny, g.nx), dtype=torch.float32, device=dev)
    gI[-1, g.ny // 2, g.nx // 2] = -1.0
    stream = torch.cuda.current_stream(dev)

    def run():
        return bpm.adjoint(u0, dn, g.dx, g.dz, g.wavelength, g.n0, grad_intensity=gI,
                           want_field=False, want_spectrum=True, want_dn=True, stream=stream)

    run()
    torch.cuda.synchronize(dev)
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        run()
        b.record(stream)
        torch.cuda.synchronize(dev)
        ts.append(a.elapsed_time(b))
    ms = float(np.median(ts))
    vs = g.nx * g.ny * g.steps
    achieved = ADJOINT_BYTES_PER_VOXEL_STEP * vs / (ms / 1e3) / 1e9

    # eight guide stars (foci at eight lateral positions of the exit plane)
    # through the same tissue, one lockstep bpm_adjoint_batch launch
    n_stars = 8
    gIs = []
    for k in range(n_stars):
        t = torch.zeros_like(gI)
        t[-1, g.ny // 2 + 8 * (k // 4) - 4, g.nx // 2 + 8 * (k % 4) - 12] = -1.0
        gIs.append(t)
    jobs = [dict(field=u0, dn=dn, grad_intensity=t, want_field=False, want_spectrum=True,
                 want_dn=True) for t in gIs]
    ws = bpm.workspace(bpm.bpm.adjoint_batch_workspace_size(n_stars, g.nx, g.ny, g.steps), dev)

    def run_batch():
        return bpm.adjoint_batch(jobs, g.dx, g.dz, g.wavelength, g.n0, ws=ws, stream=stream)

    run_batch()
    torch.cuda.synchronize(dev)
    tb = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        run_batch()
        b.record(stream)
        torch.cuda.synchronize(dev)
        tb.append(a.elapsed_time(b))
    msb = float(np.median(tb))
    achieved_b = ADJOINT_BYTES_PER_VOXEL_STEP * n_stars * vs / (msb / 1e3) / 1e9
    del ws, jobs, gIs
    return {"workload": f"adjoint {g.nx}x{g.ny}x{g.steps}, sqrt(N) checkpoints, gradients "
                        "w.r.t. pupil spectrum and dn",
            "ms": round(ms, 3), "gvoxel_steps_per_s": round(vs / (ms / 1e3) / 1e9, 3),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "bytes_per_voxel_step": ADJOINT_BYTES_PER_VOXEL_STEP},
            "lockstep": {"workload": f"{n_stars} guide stars of the same workload in one "
                                     "bpm_adjoint_batch launch",
                         "ms": round(msb, 3),
                         "gvoxel_steps_per_s": round(n_stars * vs / (msb / 1e3) / 1e9, 3),
                         "speedup_vs_separate_calls": round(n_stars * ms / msb, 2),
                         "roofline": {"bound": "hbm", "achieved": round(achieved_b, 1),
                                      "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                      "frac": round(achieved_b / HBM_PEAK_GBS, 4),
                                      "bytes_per_voxel_step": ADJOINT_BYTES_PER_VOXEL_STEP}}}


def batch_rate(dev, replays=3):
    """The uneven batch: 64 jobs, nx, ny in {256, 512, 1024}, 128-1024 steps,
    dn + intensity <= 160 GiB, one work-queue launch, timed as a replay of the
    captured device half (bpm_batch_launch in a HIP graph, the configuration
    asked for) and as a plain bpm_propagate_batch call.  dn is uniform random
    in [0, 0.05] drawn on the device (the rate does not depend on its values)."""
    import numpy as np
    import torch
    import synth
    import paper_1706_02261_amd as bpm
    from paper_1706_02261_amd import bpm as B
    specs = synth.batch_job_specs()
    gen = torch.Generator(device=dev).manual_seed(1002)
    jobs = []
    for nx, ny, steps in specs:
        u0 = torch.randn((ny, nx), dtype=torch.complex64, device=dev, generator=gen)
        dn = torch.rand((steps, ny, nx), dtype=torch.float32, device=dev, generator=gen) * 0.05
        jobs.append(dict(field=u0, dn=dn, dx=0.2, dz=0.2, wavelength=0.5, n0=1.33,
                         out=torch.empty_like(u0),
                         intensity_out=torch.empty((steps, ny, nx), dtype=torch.float32,
                                                   device=dev)))
    ws = B.workspace(B._batch_table(jobs)[2], dev)
    stream = torch.cuda.current_stream(dev)
    ev = lambda: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    bpm.propagate_batch(jobs, ws=ws, stream=stream)
    torch.cuda.synchronize(dev)
    a, b = ev()
    a.record(stream)
    bpm.propagate_batch(jobs, ws=ws, stream=stream)
    b.record(stream)
    torch.cuda.synchronize(dev)
    ms_call = a.elapsed_time(b)
    ref = [j["out"].clone() for j in jobs]
    del ws
    prep = B.PreparedBatch(jobs)
    torch.cuda.synchronize(dev)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        prep.launch()
    graph.replay()
    torch.cuda.synchronize(dev)
    ts = []
    for _ in range(replays):
        a, b = ev()
        a.record(stream)
        graph.replay()
        b.record(stream)
        torch.cuda.synchronize(dev)
        ts.append(a.elapsed_time(b))
    same = all(torch.equal(j["out"], r) for j, r in zip(jobs, ref))
    ms = float(np.median(ts))
    vs = sum(nx * ny * st for nx, ny, st in specs)
    achieved = BYTES_PER_VOXEL_STEP * vs / (ms / 1e3) / 1e9
    del jobs, prep, graph, ref
    torch.cuda.empty_cache()
    return {"workload": f"{len(specs)} uneven jobs (nx, ny in 256..1024, steps 128..1024), "
                        "one persistent work-queue launch, replayed from a captured graph",
            "voxel_steps": vs, "ms": round(ms, 2), "ms_uncaptured_call": round(ms_call, 2),
            "replay_fields_equal_call": same,
            "gvoxel_steps_per_s": round(vs / (ms / 1e3) / 1e9, 3),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "bytes_per_voxel_step": BYTES_PER_VOXEL_STEP}}


def adapted_rate(dev, field, dn, g, reps=3):
    """The march with a locally adapted expansion (each slice about its mean
    index) on the detection field of the timed volume: one field, slice means
    included, 40 B model."""
    import numpy as np
    import torch
    import paper_1706_02261_amd as bpm
    stream = torch.cuda.current_stream(dev)
    out = torch.empty_like(field)
    ws = bpm.workspace(bpm.workspace_size(g.nx, g.ny, g.steps), dev)
    run = lambda: bpm.propagate_adapted(field, dn, g.dx, g.dz, g.wavelength, g.n0,
                                        intensity=True, out=out, ws=ws, stream=stream)
    run()
    torch.cuda.synchronize(dev)
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        run()
        b.record(stream)
        torch.cuda.synchronize(dev)
        ts.append(a.elapsed_time(b))
    ms = float(np.median(ts))
    vs = g.nx * g.ny * g.steps
    gbs = BYTES_PER_VOXEL_STEP * vs / (ms / 1e3) / 1e9
    torch.cuda.empty_cache()
    return {"workload": f"adapted expansion (slice-mean reference index), detection field "
                        f"{g.nx}x{g.ny}, {g.steps} slices, intensity written",
            "ms": round(ms, 3), "gvoxel_steps_per_s": round(vs / (ms / 1e3) / 1e9, 3),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "bytes_per_voxel_step": BYTES_PER_VOXEL_STEP}}


def ao_rates(dev, reps=5):
    """Adaptive optics on the Perlin tissue (256^2 x 80, n = 1.36 +- 0.03):
    guide-star correction latency (linear adjoint + phase kernel), focus
    intensities (clear, aimed, corrected; fraction of the optimum), one Adam
    iteration of the pupil optimiser, a 12-shift memory-effect sweep, and the
    same correction through the 256^2 x 512 adjoint workload."""
    import numpy as np
    import torch
    import synth
    from paper_1706_02261_amd import ao

    def timed(fn):
        fn()
        torch.cuda.synchronize(dev)
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize(dev)
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    g, dn, amp, zf = synth.ao_workload(256, 80)
    opt = ao.Optics(g.dx, g.dz, g.wavelength, g.n0)
    f = (g.ny // 2, g.nx // 2)
    dn_t = torch.from_numpy(dn).to(dev)
    amp_t = torch.from_numpy(amp).to(dev)
    phi, gs = ao.guide_star_phase(dn_t, f, zf, opt)
    aim = ao.aim_phase(g.ny, g.nx, f, opt, device=dev)
    at = lambda ph, d: float(ao.exit_field(amp_t, ph, d, zf, opt)[f].abs() ** 2)
    corr, unc, clear = at(phi, dn_t), at(aim, dn_t), at(aim, torch.zeros_like(dn_t))
    best = ao.optimum_intensity(amp_t, gs)
    ms_gs = timed(lambda: ao.guide_star_phase(dn_t, f, zf, opt))
    prob = ao.FocusProblem(dn_t, [f])
    ms_it = timed(lambda: prob.gradient(amp_t, aim, dn_t, zf, opt))
    shifts = [(0, s) for s in range(1, 7)] + [(s, 0) for s in range(1, 7)]
    ms_me = timed(lambda: ao.memory_effect(amp_t, gs, dn_t, f, shifts, zf, opt))
    P, _ = ao.memory_effect(amp_t, gs, dn_t, f, shifts, zf, opt)
    pw = ao.plane_wave_exit(dn_t, opt)
    C = ao.speckle_autocorrelation((pw.abs() ** 2).contiguous(), 6)

    def half_width(c):
        for i in range(1, len(c)):
            if c[i] < 0.5:
                return i - 1 + (c[i - 1] - 0.5) / (c[i - 1] - c[i])
        return None
    Pm = np.r_[1.0, 0.5 * (P[:6] + P[6:])]
    g3, dn3, _, _ = synth.config3()
    dn3_t = torch.from_numpy(dn3).to(dev)
    ms_gs3 = timed(lambda: ao.guide_star_phase(dn3_t, (g3.ny // 2, g3.nx // 2),
                                               g3.steps * g3.dz, ao.Optics(g3.dx, g3.dz,
                                                                           g3.wavelength, g3.n0)))
    del dn_t, dn3_t, prob
    torch.cuda.empty_cache()
    return {"workload": "Perlin tissue 256x256x80 (dx = dz = 0.2 um, n = 1.36 +- 0.03 as a "
                        "standard deviation), NA 0.6 Gaussian pupil, focus at the exit plane",
            "mean_free_paths": round(ao.mean_free_paths(pw), 3),
            "focus_intensity": {"clear": clear, "aimed": unc, "corrected": corr,
                                "corrected_over_optimum": round(corr / best, 6),
                                "corrected_over_clear": round(corr / clear, 4),
                                "enhancement_over_aimed": round(corr / unc, 3)},
            "guide_star_ms": round(ms_gs, 4),
            "optimizer_iteration_ms": round(ms_it, 4),
            "memory_effect_sweep_ms": round(ms_me, 3), "memory_effect_shifts": len(shifts),
            "persistence_half_width_px": half_width(Pm),
            "speckle_half_width_px": half_width(C),
            "guide_star_ms_256x256x512": round(ms_gs3, 4)}


def zernike_rates(dev, dn, g, depth=512, pitch=32, n_modes=15, reps=3):
    """Aberration map of the detection volume: sources on a pitch-32 grid at
    slice `depth` (1024 sources on 1024^2), one multiplexed march to the exit
    plane, pupil fields (32 x 32 windows) and 15-mode Zernike fits; the
    time of each part (median of `reps`) and sources per second."""
    import numpy as np
    import torch
    from paper_1706_02261_amd import aberrations, psfs
    from paper_1706_02261_amd import bpm as B
    opt = psfs.Optics(g.dx, g.dz, g.wavelength, g.n0, 0.6)
    nz, ny, nx = dn.shape
    ys = torch.arange(pitch // 2, ny, pitch, dtype=torch.int32, device=dev)
    xs = torch.arange(pitch // 2, nx, pitch, dtype=torch.int32, device=dev)
    src = torch.stack(torch.meshgrid(ys, xs, indexing="ij"), -1).reshape(-1, 2).contiguous()
    ws = B.workspace(B.workspace_size(nx, ny, nz - depth), dev)
    state = {}

    def march():
        u0 = B.point_sources(src, nx, ny, opt.dx, opt.wavelength, opt.n0, opt.na, 0.0)
        state["exit"], _ = B.propagate(u0, dn[depth:], opt.dx, opt.dz, opt.wavelength, opt.n0,
                                       intensity=False, ws=ws)

    def pupils():
        state["X"] = aberrations.pupil_fields(state["exit"], src, nz - depth, opt, 32)

    def fit():
        state["c"] = aberrations.zernike_fit(state["X"], opt, n_modes)

    out = {}
    for name, fn in (("march_ms", march), ("pupil_fields_ms", pupils), ("zernike_fit_ms", fit)):
        fn()
        torch.cuda.synchronize(dev)
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize(dev)
            ts.append(a.elapsed_time(b))
        out[name] = round(float(np.median(ts)), 3)
    c, rms = state["c"]
    total = out["march_ms"] + out["pupil_fields_ms"] + out["zernike_fit_ms"]
    res = {"workload": f"{src.shape[0]} sources (pitch {pitch}) at slice {depth} of the "
                       f"{nx}x{ny}x{nz} detection volume, {nz - depth}-slice multiplexed march, "
                       f"32x32 pupil windows, {n_modes} Noll modes",
           **out, "sources_per_s": round(src.shape[0] / (total / 1e3), 1),
           "median_rms_rad": round(float(rms.median()), 4),
           "max_abs_coeff_rad": round(float(c[:, 1:].abs().max()), 3)}
    del state, ws
    torch.cuda.empty_cache()
    return res


def camera_rates(dev, dn, ls_intensity, g, half_depth=15, pitch=32, reps=2):
    """One camera frame of the detection volume focused on its middle slice:
    excitation from the timed light-sheet march (its intensity volume, back in
    the detection frame), fluorophores where dn > 0.01, node PSFs on a pitch-32
    grid at the 31 depths around focus (uneven batch marches of 8 depths, one
    refocus readout each) and the spatially varying sum."""
    import numpy as np
    import torch
    from paper_1706_02261_amd import imaging, psfs
    opt = psfs.Optics(g.dx, g.dz, g.wavelength, g.n0, 0.6)
    nz, ny, nx = dn.shape
    f = nz // 2
    exc = ls_intensity.permute(2, 1, 0).contiguous()     # [x][y][z] -> [z][y][x]
    dens = (dn > 0.01).to(torch.float32)
    run = lambda: imaging.camera_image(exc, dens, dn, f, pitch, opt, half_depth=half_depth)
    img = run()
    torch.cuda.synchronize(dev)
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        img = run()
        b.record()
        torch.cuda.synchronize(dev)
        ts.append(a.elapsed_time(b))
    ms = float(np.median(ts))
    # the image sum alone: 31 slabs through one depth's node PSFs
    P = torch.rand((ny // pitch, nx // pitch, 32, 32), device=dev)
    acc = torch.zeros((ny, nx), dtype=torch.float32, device=dev)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for z in range(2 * half_depth + 1):
        imaging.camera_accumulate(acc, exc[f], P, pitch, density=dens[f])
    b.record()
    torch.cuda.synchronize(dev)
    sum_ms = a.elapsed_time(b)
    depths = 2 * half_depth + 1
    n_psf = depths * (ny // pitch) * (nx // pitch)
    # 32 x 32 PSF taps over ~9 nodes per output pixel (hat supports overlap)
    macs = depths * nx * ny * 32 * 32 * 9
    res = {"workload": f"{nx}x{ny} camera frame focused on slice {f} of the {nx}x{ny}x{nz} "
                       f"volume: {depths} depths x {(ny // pitch) * (nx // pitch)} node PSFs "
                       f"(pitch {pitch}), light-sheet excitation, fluorophores where dn > 0.01",
           "frame_ms": round(ms, 2), "psfs_per_s": round(n_psf / (ms / 1e3), 1),
           "image_sum_ms": round(sum_ms, 3),
           "image_sum_fp32_tflops": round(2 * macs / (sum_ms / 1e3) / 1e12, 2),
           "image_mean": round(float(img.mean()), 4)}
    del exc, dens, P, acc, img
    torch.cuda.empty_cache()
    return res


def phase_split(jobs, ws, stream, launch_ms):
    """One run of the timed launch with per-workgroup phase timers: mean and
    max over workgroups of each phase, in microseconds per step."""
    import torch
    from paper_1706_02261_amd import bpm as B
    _, t = B.march_phase_times(jobs, ws=ws, stream=stream)
    torch.cuda.synchronize()
    steps = t["steps"]
    out = {"workgroups": t["workgroups"], "fields": t["fields"], "steps": steps,
           "unit": "us per step (mean over workgroups / max)",
           "launch_us_per_step": round(launch_ms * 1e3 / steps, 3)}
    for name in B.PHASES:
        v = t[name] * 1e6 / steps
        out[name] = [round(float(v.mean()), 3), round(float(v.max()), 3)]
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed marches")
    ap.add_argument("--warmup", type=int, default=2, help="untimed marches")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--slices", type=int, default=1024, help="march depth (default 1024)")
    ap.add_argument("--no-psf", action="store_true", help="skip the surrogate vs BPM PSF rates")
    ap.add_argument("--train-seconds", type=float, default=60.0,
                    help="surrogate training time of the PSF block (default 60)")
    ap.add_argument("--psf-only", action="store_true",
                    help="only the surrogate vs BPM PSF rates (for profiling those kernels)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the uneven-batch rate (for profiling the work-queue kernel)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the adjoint and uneven-batch rates")
    ap.add_argument("--tune", action="store_true",
                    help="time every kernel the march offers for the benchmark's shape first, "
                         "keep the fastest (launch-shape tuner) and record it in the cache")
    ap.add_argument("--phase-times", action="store_true",
                    help="also run the timed launch once with per-workgroup phase timers and "
                         "report the split of a step into pass work, store drain and barrier "
                         "waits")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (the known-size "
                         "kernel that scales rocprofv3's FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} (WORLD_SIZE "
              f"{world}) is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1706_02261_amd as bpm
    from paper_1706_02261_amd import bpm as B
    import synth

    dev = torch.device("cuda:0")
    if args.psf_only:
        print(json.dumps({"metric": "surrogate vs BPM PSFs/s",
                          "psf": psf_rates(dev, train_seconds=args.train_seconds)}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"metric": "uneven batch Gvoxel-steps/s",
                          "uneven_batch": batch_rate(dev, replays=1)}), flush=True)
        return
    t_gen = time.perf_counter()
    g, u0, dn_host = synth.config2_detection(steps=args.slices)
    gl, u0_ls, dn_ls = synth.config2_light_sheet(g, dn_host)
    t_gen = time.perf_counter() - t_gen
    if (gl.nx, gl.ny, gl.steps, gl.dx, gl.dz) != (g.nx, g.ny, g.steps, g.dx, g.dz):
        sys.exit("bench.py: the light-sheet march must have the detection march's geometry")
    field = torch.from_numpy(u0).to(dev)
    dn = torch.from_numpy(dn_host).to(dev)
    jobs = []
    for f, d in ((field, dn), (torch.from_numpy(u0_ls).to(dev), torch.from_numpy(dn_ls).to(dev))):
        jobs.append(dict(field=f, dn=d, dx=g.dx, dz=g.dz, wavelength=g.wavelength, n0=g.n0,
                         out=torch.empty_like(f),
                         intensity_out=torch.empty((g.steps, g.ny, g.nx), dtype=torch.float32,
                                                   device=dev)))
    del dn_ls
    arr = (B._lib.Job * 2)(*[B._lib.Job(j["field"].data_ptr(), j["dn"].data_ptr(), g.nx, g.ny,
                                        g.steps, g.dx, g.dz, g.wavelength, g.n0,
                                        j["out"].data_ptr(), j["intensity_out"].data_ptr())
                             for j in jobs])
    ws = B.workspace(B.lib().bpm_batch_workspace_size(arr, 2), dev)
    stream = torch.cuda.current_stream(dev)
    from paper_1706_02261_amd import tune
    tuned = tune.tune([(g.nx, g.ny, len(jobs))], steps=16) if args.tune else None
    if tuned:
        tune.save(tuned)
    else:
        tune.load()
    variant = tune.VARIANTS[tune.current_variant(g.nx, g.ny, len(jobs))]

    def march():
        bpm.propagate_batch(jobs, ws=ws, stream=stream)

    for _ in range(args.warmup):
        march()
    torch.cuda.synchronize(dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        march()
        b.record(stream)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    per_launch_ms = [a.elapsed_time(b) for a, b in ev]
    ms = wall * 1e3 / args.steps
    launch_ms = float(np.mean(per_launch_ms))
    voxel_steps = len(jobs) * g.nx * g.ny * g.steps
    value = voxel_steps / (ms / 1e3) / 1e9
    achieved = BYTES_PER_VOXEL_STEP * voxel_steps / (launch_ms / 1e3) / 1e9
    traffic_bytes = measured_traffic()
    traffic = None if traffic_bytes is None else round(traffic_bytes / (launch_ms / 1e3) / 1e9, 1)
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gvoxel-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": round(value / PAPER_GVS, 2),
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"paper-scale step: the detection march ({g.nx}x{g.ny} complex64 "
                        f"field, {g.steps} slices, 1000 multiplexed NA 0.6 point sources) and "
                        "the light-sheet march (NA 0.15, same volume permuted z<->x) through an "
                        "embryo-like ellipsoid phantom (n 1.33-1.38), dx=dz=0.2 um, "
                        "lambda=0.5 um, n0=1.33, both intensity volumes written, one "
                        "lockstep launch",
            "nx": g.nx, "ny": g.ny, "slices": g.steps, "fields": len(jobs), "sources": 1000,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_bytes_per_voxel_step": None if traffic_bytes is None
            else round(traffic_bytes / voxel_steps, 2),
            "kernel": f"march ({variant} kernel), 2 fields in one launch per step, plan "
                      "kernel included",
            "launch_variant": variant,
            "tuner_ms": None if not tuned else next(iter(tuned.values()))["ms"],
            "launch_ms": round(launch_ms, 4),
            "bytes_per_voxel_step": BYTES_PER_VOXEL_STEP,
            "fp32_tflops": round(FLOP_PER_VOXEL_STEP * voxel_steps / (launch_ms / 1e3) / 1e12, 2),
            "fp32_frac": round(FLOP_PER_VOXEL_STEP * voxel_steps / (launch_ms / 1e3) / 1e12
                               / FP32_PEAK_TFLOPS, 4),
        },
        "input_generation_s": round(t_gen, 1),
    }
    if args.phase_times:
        line["phase_split"] = phase_split(jobs, ws, stream, launch_ms)
    if args.copy_mib:
        src = torch.ones(args.copy_mib * 2 ** 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize(dev)
        line["copy_calibration_bytes"] = src.numel() * 4
    if not args.no_psf:
        line["psf"] = psf_rates(dev, train_seconds=args.train_seconds)
    small = None
    if not (args.no_extra and args.no_cpu_baseline):
        small = {"128x128x64": synth.config0(), "512x512x512": synth.config1()}
        g1, _, dn1 = small["512x512x512"]
        # the same volume lit by a bound hexagonal Bessel lattice (NA 0.55 / 0.45)
        small["512x512x512_bessel_lattice"] = (
            g1, synth.bessel_lattice_field(g1.nx, g1.ny, g1.dx, g1.wavelength, g1.n0, 0.55,
                                           0.45, 6, (0.08, 0.01)), dn1)
    if not args.no_extra:
        line["workloads"] = workload_rates(dev, small)
        line["adapted"] = adapted_rate(dev, jobs[0]["field"], jobs[0]["dn"], g)
        line["adjoint"] = adjoint_rate(dev)
        line["adaptive_optics"] = ao_rates(dev)
        line["zernike_map"] = zernike_rates(dev, jobs[0]["dn"], g, depth=g.steps // 2)
        line["camera_frame"] = camera_rates(dev, jobs[0]["dn"], jobs[1]["intensity_out"], g)
        line["uneven_batch"] = batch_rate(dev)
    if not args.no_cpu_baseline:
        def gpu_first(steps):
            # the timed launch's configuration (both fields in lockstep), cut to the sample
            part = [dict(j, dn=j["dn"][:steps], out=None, intensity_out=None, intensity=False)
                    for j in jobs]
            (o, _), _ = bpm.propagate_batch(part)
            torch.cuda.synchronize(dev)
            return o.cpu().numpy()
        line["cpu_baseline"] = cpu_baseline(u0, dn_host, g, gpu_first, small)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
