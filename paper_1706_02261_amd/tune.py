"""Launch-shape tuner of the forward march.

For each shape (nx, ny, lockstep fields) the library offers one or more
kernels (include/bpm.h, BPM_MARCH_*): one workgroup per CU with register
twiddles, two per CU with LDS twiddles, the tiled march of one or two fields, and
64-thread workgroups for small fields.  They
give identical results; which is fastest depends on the shape and the device.
``tune`` times every eligible kernel of each shape on the current device (a
short march of random fields, median of a few launches timed with events on
the launch stream) and records the fastest with ``bpm_set_march_variant``;
``save``/``load`` keep the choices in a JSON file per device name and CU
count, so a later process applies them without timing again.

Cache file: $BPM_TUNING_FILE, else ~/.cache/paper_1706_02261_amd/march_variants.json.
"""
from __future__ import annotations

import json
import os

import torch

from . import _lib
from . import bpm as _bpm
from ._lib import check, lib

VARIANTS = {_lib.BPM_MARCH_ONE_PER_CU: "one_per_cu", _lib.BPM_MARCH_TWO_PER_CU: "two_per_cu",
            _lib.BPM_MARCH_TILED_PAIR: "tiled_pair", _lib.BPM_MARCH_SMALL_BLOCKS: "small_blocks"}


def cache_path() -> str:
    return os.environ.get("BPM_TUNING_FILE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_1706_02261_amd", "march_variants.json")


def device_key(device) -> str:
    p = torch.cuda.get_device_properties(device)
    return f"{p.name}/{p.multi_processor_count}cu"


def eligible(nx: int, ny: int, fields: int):
    return [v for v in VARIANTS if lib().bpm_march_variant_eligible(nx, ny, fields, v)]


def set_variant(nx: int, ny: int, fields: int, variant: int) -> None:
    check(lib().bpm_set_march_variant(nx, ny, fields, variant), "bpm_set_march_variant")


def current_variant(nx: int, ny: int, fields: int) -> int:
    v = lib().bpm_march_variant(nx, ny, fields)
    check(v if v < 0 else 0, "bpm_march_variant")
    return v


def _time(jobs, reps: int, stream) -> float:
    ws = _bpm.workspace(_bpm._batch_table(jobs)[2], jobs[0]["field"].device)
    run = (lambda: _bpm.propagate_batch(jobs, ws=ws, stream=stream))
    run()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        run()
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def tune(shapes, steps: int = 32, reps: int = 5, device="cuda", stream=None, seed: int = 0):
    """Time every eligible kernel of each (nx, ny, fields) shape and keep the
    fastest.  Returns {(nx, ny, fields): {"variant": v, "ms": {name: ms}}}."""
    dev = torch.device(device)
    s = torch.cuda.current_stream(dev) if stream is None else stream
    g = torch.Generator(device=dev).manual_seed(seed)
    out = {}
    for nx, ny, fields in shapes:
        jobs = [dict(field=torch.randn((ny, nx), dtype=torch.complex64, device=dev, generator=g),
                     dn=torch.rand((steps, ny, nx), device=dev, generator=g) * 0.05,
                     dx=0.2, dz=0.2, wavelength=0.5, n0=1.33, intensity=True)
                for _ in range(fields)]
        ms = {}
        for v in eligible(nx, ny, fields):
            set_variant(nx, ny, fields, v)
            ms[v] = _time(jobs, reps, s)
        best = min(ms, key=ms.get)
        set_variant(nx, ny, fields, best)
        out[(nx, ny, fields)] = {"variant": best,
                                 "ms": {VARIANTS[v]: round(t, 4) for v, t in ms.items()}}
        del jobs
    return out


def save(results, device="cuda", path: str | None = None) -> str:
    """Merge tuning results into the JSON cache under this device's key."""
    path = path or cache_path()
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    entries = data.setdefault(device_key(torch.device(device)), {})
    for (nx, ny, fields), r in results.items():
        entries[f"{nx}x{ny}x{fields}"] = {"variant": VARIANTS[r["variant"]], "ms": r["ms"]}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return path


def load(device="cuda", path: str | None = None) -> dict:
    """Apply the cached choices of this device (entries of other devices and
    choices the current build cannot run are skipped).  Returns those applied."""
    path = path or cache_path()
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        entries = json.load(f).get(device_key(torch.device(device)), {})
    names = {n: v for v, n in VARIANTS.items()}
    applied = {}
    for key, r in entries.items():
        nx, ny, fields = (int(t) for t in key.split("x"))
        v = names.get(r.get("variant"))
        if v is not None and v in eligible(nx, ny, fields):
            set_variant(nx, ny, fields, v)
            applied[(nx, ny, fields)] = v
    return applied
