"""Spatially varying PSFs from the BPM and from the learned surrogate.

The BPM definition (main text, paragraphs on multiplexing and on the
detection path): point sources at one depth d of a dn volume with nz slices
ride in one multiplexed field, which is marched through slices d … nz-1 and
read out through the idealised refocusing lens (bpm_psf_readout, 32 planes of
spacing dz around the source plane, 32 x 32 crops).  Stacks are scaled by
1 / (peak of the same readout in a dn = 0 medium), so a clear-medium PSF
peaks at 1.

The surrogate (psf_surrogate_infer) predicts the same stack from the
[64][32][32] dn patch around the source and its depth, together with its own
relative error; ``psf_with_fallback`` replaces every prediction whose error
estimate exceeds the threshold by the BPM stack.

Orchestration only: every array operation runs in libbpm.so.
"""
from __future__ import annotations

import dataclasses

import torch

from . import bpm as _bpm
from . import surrogate as _sg
from .bpm import _need

PLANES = 32
CROP = 32


@dataclasses.dataclass(frozen=True)
class Optics:
    """Sampling and optics of the PSF volume (lengths in micrometres)."""
    dx: float = 0.2
    dz: float = 0.2
    wavelength: float = 0.5
    n0: float = 1.33
    na: float = 0.6


def reference_peak(nx: int, ny: int, optics: Optics = Optics(), device="cuda") -> float:
    """Peak of the dn = 0 PSF stack: the readout of one in-focus source with no
    medium to cross (free-space propagation composes exactly)."""
    src = torch.tensor([[ny // 2, nx // 2]], dtype=torch.int32, device=device)
    u0 = _bpm.point_sources(src, nx, ny, optics.dx, optics.wavelength, optics.n0, optics.na, 0.0)
    psf = _bpm.psf_readout(u0, src, optics.dx, optics.dz, optics.wavelength, optics.n0,
                           optics.na, 0, planes=PLANES, crop=CROP)
    return float(psf.max())


def bpm_psfs(dn: torch.Tensor, depth: int, sources: torch.Tensor, scale: float,
             optics: Optics = Optics(), ws=None, out: torch.Tensor | None = None):
    """BPM PSF stacks [n][32][32][32] of point sources at slice ``depth`` of
    ``dn`` [nz][ny][nx] (``sources`` int32 [n][2] (y, x), one multiplexed run)."""
    _need(dn, "dn", torch.float32)
    nz, ny, nx = dn.shape
    if not 0 <= depth < nz:
        raise ValueError(f"depth={depth} must be in [0, {nz})")
    u0 = _bpm.point_sources(sources, nx, ny, optics.dx, optics.wavelength, optics.n0, optics.na,
                            0.0)
    exit_field, _ = _bpm.propagate(u0, dn[depth:], optics.dx, optics.dz, optics.wavelength,
                                   optics.n0, intensity=False, ws=ws)
    psf = _bpm.psf_readout(exit_field, sources, optics.dx, optics.dz, optics.wavelength,
                           optics.n0, optics.na, nz - depth, planes=PLANES, crop=CROP,
                           scale=scale)
    if out is not None:
        out.copy_(psf)
        return out
    return psf


def training_run(dn: torch.Tensor, depth: int, offset, pitch: int, scale: float,
                 optics: Optics = Optics()):
    """One multiplexed run of the training-set generator: sources on a
    ``pitch`` grid shifted by ``offset`` (y, x) at slice ``depth`` of a 64-slice
    volume.  Returns (patches [n][64][32][32], depth [n], PSFs [n][32][32][32])."""
    nz, ny, nx = dn.shape
    if nz != _sg.PATCH[0]:
        raise ValueError(f"the surrogate's volumes have {_sg.PATCH[0]} slices, got {nz}")
    dev = dn.device
    ys = torch.arange(offset[0] % pitch, ny, pitch, dtype=torch.int32, device=dev)
    xs = torch.arange(offset[1] % pitch, nx, pitch, dtype=torch.int32, device=dev)
    src = torch.stack(torch.meshgrid(ys, xs, indexing="ij"), -1).reshape(-1, 2).contiguous()
    patches = _sg.extract_patches(dn, src, 0)
    dep = torch.full((src.shape[0],), float(depth), dtype=torch.float32, device=dev)
    return patches, dep, bpm_psfs(dn, depth, src, scale, optics)


def fallback_runs(yx, ny: int, nx: int, min_separation: int = CROP):
    """Split sources ((y, x) pixels, host int array [n][2]) into multiplexed
    runs in which every two sources lie more than ``min_separation`` pixels
    apart along y or x (circularly): a stack then sees neighbours no closer
    than in the training runs, whose sources sit on a grid of that pitch.

    The plane is cut into square cells of side P (the power of two >=
    min_separation, at most the field's side); cells are coloured by the
    parity of their row and column index (a third colour for the last cell of
    an odd count, which wraps onto cell 0), and the k-th source of a cell goes
    to run (colour, k).  Two sources of one run are therefore in different
    cells of one colour, at least one full cell apart.  Returns a list of
    index arrays, one per run."""
    import numpy as np
    yx = np.asarray(yx, dtype=np.int64).reshape(-1, 2)
    if len(yx) == 0:
        return []

    def axis(v, n):
        P = 1
        while P < min(max(min_separation, 1), n):
            P *= 2
        P = min(P, n)
        c = (v % n) // P
        nc = n // P
        col = c % 2
        if nc % 2 == 1 and nc > 1:
            col = np.where(c == nc - 1, 2, col)
        return c, col, nc

    cy, coly, ncy = axis(yx[:, 0], ny)
    cx, colx, ncx = axis(yx[:, 1], nx)
    cell = cy * ncx + cx
    order = np.argsort(cell, kind="stable")
    rank = np.empty(len(yx), dtype=np.int64)
    sc = cell[order]
    start = np.r_[0, np.nonzero(np.diff(sc))[0] + 1]
    first = np.repeat(start, np.diff(np.r_[start, len(sc)]))
    rank[order] = np.arange(len(sc)) - first
    key = (coly * 3 + colx) * (int(rank.max()) + 1) + rank
    return [np.nonzero(key == k)[0] for k in np.unique(key)]


def psf_with_fallback(weights: torch.Tensor, dn: torch.Tensor, sources: torch.Tensor,
                      scale: float, threshold: float = 0.05, optics: Optics = Optics(),
                      min_separation: int = CROP):
    """PSF stacks of point sources (int32 [n][3] = (z, y, x)) in a 64-slice
    volume: the surrogate's prediction, or the BPM stack where the predicted
    relative error exceeds ``threshold``.

    Returns (psf [n][32][32][32], pred_err [n], fallback mask [n] bool).  The
    flagged sources of each depth are split into runs (``fallback_runs``) so
    that no two sources of one multiplexed march lie within
    ``min_separation`` pixels of each other; a depth's runs march together,
    up to eight in one lockstep launch, and each is read out on its own, so a
    replaced stack is bitwise the BPM readout of its run."""
    import numpy as np
    _need(dn, "dn", torch.float32)
    _need(sources, "sources", torch.int32)
    if sources.dim() != 2 or sources.shape[1] != 3:
        raise ValueError("sources must be [n][3] (z, y, x)")
    nz, ny, nx = dn.shape
    if nz != _sg.PATCH[0]:
        raise ValueError(f"the surrogate's volumes have {_sg.PATCH[0]} slices, got {nz}")
    yx = sources[:, 1:].contiguous()
    depth = sources[:, 0].to(torch.float32).contiguous()
    patches = _sg.extract_patches(dn, yx, 0)
    psf, err = _sg.infer(weights, patches, depth)
    flagged = err > threshold
    idx = torch.nonzero(flagged).flatten()
    if idx.numel():
        src_h = sources[idx].cpu().numpy()
        idx_h = idx.cpu().numpy()
        for d in np.unique(src_h[:, 0]).tolist():
            at = np.nonzero(src_h[:, 0] == d)[0]
            runs = [at[r] for r in fallback_runs(src_h[at, 1:], ny, nx, min_separation)]
            for b in range(0, len(runs), _MAX_LOCKSTEP):
                group = runs[b:b + _MAX_LOCKSTEP]
                sel = [torch.from_numpy(idx_h[r]).to(psf.device) for r in group]
                stacks = _bpm_psfs_runs(dn, int(d), [yx[s_].contiguous() for s_ in sel], scale,
                                        optics)
                for s_, st in zip(sel, stacks):
                    psf[s_] = st
    return psf, err, flagged


_MAX_LOCKSTEP = 8   # fields of one geometry that march in one lockstep launch


def _bpm_psfs_runs(dn: torch.Tensor, depth: int, runs, scale: float, optics: Optics):
    """bpm_psfs of several runs at one depth, their marches in one batch call."""
    nz, ny, nx = dn.shape
    jobs = []
    for src in runs:
        u0 = _bpm.point_sources(src, nx, ny, optics.dx, optics.wavelength, optics.n0, optics.na,
                                0.0)
        jobs.append(dict(field=u0, dn=dn[depth:], dx=optics.dx, dz=optics.dz,
                         wavelength=optics.wavelength, n0=optics.n0, out=u0, intensity=False))
    exits = _bpm.propagate_batch(jobs)
    return [_bpm.psf_readout(o, src, optics.dx, optics.dz, optics.wavelength, optics.n0,
                             optics.na, nz - depth, planes=PLANES, crop=CROP, scale=scale)
            for (o, _), src in zip(exits, runs)]
