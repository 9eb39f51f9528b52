"""Camera images of a fluorescent object (Fig. 1c; main-text paragraph on the
light-sheet simulation).

The detection objective is focused on slice ``focal_slice`` of a dn volume.
For every depth z of a slab around it, point sources on a pitch grid at
depth z ride in one multiplexed field, march to the exit plane (the depths in
lockstep launches of equal-length jobs, see ``focal_plane_psfs``) and are
brought back through the detection pupil to the focal plane (``bpm_psf_readout`` with one plane, back_steps = nz -
focal_slice); their crops are the node PSFs of that depth in the camera
plane.  ``bpm_camera_accumulate`` then adds the depth's emission
(excitation x fluorophore density) through the node PSFs, blended
bilinearly between nodes.  Depths beyond the slab contribute nothing (their
blur falls outside the readout window).

Orchestration only: marches, readouts and the image sum run in libbpm.so.
"""
from __future__ import annotations

import torch

from . import bpm as _bpm
from ._lib import check, lib
from .bpm import _need, _ptr, _stream_ptr
from .psfs import Optics, reference_peak


def node_sources(ny: int, nx: int, pitch: int, device) -> torch.Tensor:
    """int32 [gy * gx][2] node pixels (pitch/2 + pitch i, pitch/2 + pitch j)."""
    ys = torch.arange(pitch // 2, ny, pitch, dtype=torch.int32, device=device)
    xs = torch.arange(pitch // 2, nx, pitch, dtype=torch.int32, device=device)
    return torch.stack(torch.meshgrid(ys, xs, indexing="ij"), -1).reshape(-1, 2).contiguous()


def camera_accumulate(image: torch.Tensor, excitation: torch.Tensor, node_psfs: torch.Tensor,
                      pitch: int, density: torch.Tensor | None = None, stream=None):
    """image [ny][nx] += the slab's emission through the node PSFs
    [ny/pitch][nx/pitch][crop][crop] (in place; returns image)."""
    _need(image, "image", torch.float32)
    ny, nx = image.shape
    _need(excitation, "excitation", torch.float32, (ny, nx))
    if density is not None:
        _need(density, "density", torch.float32, (ny, nx))
    _need(node_psfs, "node_psfs", torch.float32)
    crop = node_psfs.shape[-1]
    if tuple(node_psfs.shape) != (ny // pitch, nx // pitch, crop, crop):
        raise ValueError(f"node_psfs has shape {tuple(node_psfs.shape)}, expected "
                         f"[{ny // pitch}][{nx // pitch}][crop][crop]")
    rc = lib().bpm_camera_accumulate(_ptr(excitation), _ptr(density), _ptr(node_psfs), nx, ny,
                                     int(pitch), int(crop), _ptr(image), _stream_ptr(stream))
    check(rc, "bpm_camera_accumulate")
    return image


def focal_plane_psfs(dn: torch.Tensor, depths, focal_slice: int, pitch: int,
                     optics: Optics = Optics(), crop: int = 32, scale: float = 1.0):
    """Node PSFs [len(depths)][gy][gx][crop][crop] in the focal plane of
    sources at each depth, one readout per depth.  All depths march from the
    shallowest one, z0: the sources of depth z enter as the clear-medium
    field that focuses (z - z0) dz downstream and skip the screens of slices
    z0 .. z - 1 (``clear_steps``), which leaves the volume exactly as a march
    from z; the jobs then have one length and march in lockstep."""
    _need(dn, "dn", torch.float32)
    nz, ny, nx = dn.shape
    if not 0 <= focal_slice <= nz:
        raise ValueError(f"focal_slice={focal_slice} must be in [0, {nz}]")
    src = node_sources(ny, nx, pitch, dn.device)
    for z in depths:
        if not 0 <= z < nz:
            raise ValueError(f"depth {z} outside [0, {nz})")
    z0 = min(depths)
    jobs = []
    for z in depths:
        u0 = _bpm.point_sources(src, nx, ny, optics.dx, optics.wavelength, optics.n0, optics.na,
                                (z - z0) * optics.dz)
        jobs.append(dict(field=u0, dn=dn[z0:], dx=optics.dx, dz=optics.dz,
                         wavelength=optics.wavelength, n0=optics.n0, out=u0, intensity=False,
                         clear_steps=z - z0))
    exits = _bpm.propagate_batch(jobs)
    gy, gx = ny // pitch, nx // pitch
    out = torch.empty((len(jobs), gy, gx, crop, crop), dtype=torch.float32, device=dn.device)
    for k, (o, _) in enumerate(exits):
        psf = _bpm.psf_readout(o, src, optics.dx, optics.dz, optics.wavelength, optics.n0,
                               optics.na, nz - focal_slice, planes=1, crop=crop, scale=scale)
        out[k] = psf.reshape(gy, gx, crop, crop)
    return out


def camera_image(excitation: torch.Tensor, density: torch.Tensor, dn: torch.Tensor,
                 focal_slice: int, pitch: int = 32, optics: Optics = Optics(),
                 half_depth: int = 15, crop: int = 32, batch: int = 8):
    """Camera image [ny][nx] with the detection focused on ``focal_slice``:
    the emission excitation x density ([nz][ny][nx] each) of the depths
    focal_slice - half_depth .. focal_slice + half_depth (clipped to the
    volume) through that depth's node PSFs.  PSFs are scaled so that a
    clear-medium PSF peaks at 1.  Depths are marched ``batch`` at a time."""
    _need(excitation, "excitation", torch.float32)
    _need(density, "density", torch.float32, tuple(excitation.shape))
    _need(dn, "dn", torch.float32, tuple(excitation.shape))
    nz, ny, nx = dn.shape
    scale = 1.0 / reference_peak(nx, ny, optics, device=dn.device)
    image = torch.zeros((ny, nx), dtype=torch.float32, device=dn.device)
    depths = list(range(max(0, focal_slice - half_depth), min(nz, focal_slice + half_depth + 1)))
    for b in range(0, len(depths), batch):
        part = depths[b:b + batch]
        P = focal_plane_psfs(dn, part, focal_slice, pitch, optics, crop, scale)
        for k, z in enumerate(part):
            camera_accumulate(image, excitation[z], P[k], pitch, density=density[z])
    return image
