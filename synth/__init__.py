"""Seeded synthetic inputs for the beam-propagation march.

This module builds inputs only: refractive-index phantoms, source fields
(single and multiplexed point sources, a cylindrical light sheet, Bessel
beams and Bessel lattices) and the
job tables of uneven batches.  It holds none of the march's arithmetic (no
propagator, no phase screen, no FFT of the march) and imports neither the
CPU oracle nor the GPU package, so that both can be fed from it.

Physical conventions (all lengths in micrometres, wavelength in vacuum):

* lateral voxel centres  x_i = (i - N/2) * dx, square pixels (dy = dx);
* axial voxel centres    z_j = (j + 1/2) * dz, one dn slice per march step;
* dn = n - n0 with the background index n0 (1.33, water);
* a field is complex64 ``[ny][nx]`` with x fastest.

The paper's phantoms are not available; every generator below is a stand-in
with the shapes and index ranges the paper reports (n = 1.33-1.38 for the
multicellular phantom of Fig. 1a, n = 1.35-1.39 for the embryo model of
Fig. 2a, n = 1.36 +- 0.03 for the Perlin-noise tissue of Fig. 2c).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "rng", "lateral_coords", "axial_coords", "add_spheres", "sphere_phantom",
    "smoothed_noise", "point_source_spectrum", "point_source_field",
    "multiplexed_field", "jittered_grid", "light_sheet_field", "Geometry",
    "bessel_spectrum", "bessel_field", "lattice_spectrum", "bessel_lattice_field",
    "perlin_noise", "perlin_phantom", "ao_workload", "fluorophore_density",
    "config0", "config1", "config2_detection", "config2_light_sheet",
    "config3", "batch_job_specs", "ellipsoid_phantom", "surrogate_volume",
]


# ---------------------------------------------------------------------------
# seeds

def rng(config_index: int, child: int = 0) -> np.random.Generator:
    """Generator for sub-part ``child`` of workload ``config_index``.

    Seeds are ``SeedSequence(1000 + config_index)`` with spawned children, so
    each sub-part (phantom, sources, phases, ...) has its own stream.
    """
    ss = np.random.SeedSequence(1000 + int(config_index))
    return np.random.default_rng(ss.spawn(int(child) + 1)[int(child)])


@dataclasses.dataclass(frozen=True)
class Geometry:
    """Grid and optics of one march (lengths in micrometres)."""
    nx: int
    ny: int
    steps: int
    dx: float
    dz: float
    wavelength: float = 0.5
    n0: float = 1.33


# ---------------------------------------------------------------------------
# coordinates

def lateral_coords(n: int, d: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) - n / 2) * d


def axial_coords(nz: int, dz: float) -> np.ndarray:
    return (np.arange(nz, dtype=np.float64) + 0.5) * dz


# ---------------------------------------------------------------------------
# phantoms

def add_spheres(dn: np.ndarray, dx: float, dz: float, centers, radii, values) -> None:
    """Paint spheres into ``dn[z][y][x]`` in place; overlaps keep the maximum.

    A voxel belongs to a sphere when its centre lies at distance <= radius.
    Centres are in the coordinates of ``lateral_coords``/``axial_coords``.
    """
    nz, ny, nx = dn.shape
    xs = lateral_coords(nx, dx)
    ys = lateral_coords(ny, dx)
    zs = axial_coords(nz, dz)
    for (cz, cy, cx), r, v in zip(centers, radii, values):
        i0 = max(0, int(math.floor((cx - r) / dx + nx / 2)))
        i1 = min(nx, int(math.ceil((cx + r) / dx + nx / 2)) + 1)
        j0 = max(0, int(math.floor((cy - r) / dx + ny / 2)))
        j1 = min(ny, int(math.ceil((cy + r) / dx + ny / 2)) + 1)
        k0 = max(0, int(math.floor((cz - r) / dz - 0.5)))
        k1 = min(nz, int(math.ceil((cz + r) / dz - 0.5)) + 1)
        if i0 >= i1 or j0 >= j1 or k0 >= k1:
            continue
        d2 = ((zs[k0:k1, None, None] - cz) ** 2
              + (ys[None, j0:j1, None] - cy) ** 2
              + (xs[None, None, i0:i1] - cx) ** 2)
        block = dn[k0:k1, j0:j1, i0:i1]
        np.maximum(block, np.where(d2 <= r * r, np.float32(v), np.float32(0)), out=block)


def sphere_phantom(g: Geometry, n_spheres: int, r_range, dn_range,
                   gen: np.random.Generator, dtype=np.float32) -> np.ndarray:
    """Random spheres, centres uniform in the volume, radius and dn uniform."""
    dn = np.zeros((g.steps, g.ny, g.nx), dtype=dtype)
    lx, ly, lz = g.nx * g.dx, g.ny * g.dx, g.steps * g.dz
    cx = gen.uniform(-lx / 2, lx / 2, n_spheres)
    cy = gen.uniform(-ly / 2, ly / 2, n_spheres)
    cz = gen.uniform(0.0, lz, n_spheres)
    r = gen.uniform(r_range[0], r_range[1], n_spheres)
    v = gen.uniform(dn_range[0], dn_range[1], n_spheres)
    add_spheres(dn, g.dx, g.dz, zip(cz, cy, cx), r, v)
    return dn


def smoothed_noise(shape, sigma_vox: float, std: float, gen: np.random.Generator,
                   coarse: int = 1) -> np.ndarray:
    """White noise smoothed by a Gaussian of ``sigma_vox`` voxels, rescaled to ``std``.

    With ``coarse > 1`` the noise is drawn and smoothed on a grid ``coarse``
    times coarser in every axis and brought back by periodic linear
    interpolation; this keeps 1024^3 volumes cheap to build on the host while
    keeping the correlation length.
    """
    from scipy import ndimage
    shape = tuple(int(s) for s in shape)
    if coarse > 1:
        cshape = tuple(max(1, s // coarse) for s in shape)
        c = gen.standard_normal(cshape).astype(np.float32)
        c = ndimage.gaussian_filter(c, sigma_vox / coarse, mode="wrap")
        out = c
        for axis, n in enumerate(shape):
            out = _lin_upsample(out, axis, n)
    else:
        out = gen.standard_normal(shape).astype(np.float32)
        out = ndimage.gaussian_filter(out, sigma_vox, mode="wrap")
    s = float(out.std())
    out *= np.float32(std / s if s > 0 else 0.0)
    return out.astype(np.float32, copy=False)


def _lin_upsample(a: np.ndarray, axis: int, n: int) -> np.ndarray:
    m = a.shape[axis]
    if m == n:
        return a
    pos = (np.arange(n, dtype=np.float64) + 0.5) * m / n - 0.5
    i0 = np.floor(pos).astype(np.int64)
    w = (pos - i0).astype(np.float32)
    i0m = i0 % m
    i1m = (i0 + 1) % m
    a0 = np.take(a, i0m, axis=axis)
    a1 = np.take(a, i1m, axis=axis)
    shp = [1] * a.ndim
    shp[axis] = n
    w = w.reshape(shp)
    return a0 * (1 - w) + a1 * w


def ellipsoid_phantom(g: Geometry, semi_axes, n_cells: int, gen: np.random.Generator,
                      base_dn=0.01, cell_r=(3.0, 5.0), cell_dn=(0.01, 0.04),
                      noise_std=0.005, noise_sigma_um=1.0, clip=(0.0, 0.05)) -> np.ndarray:
    """Embryo-like ellipsoid: interior dn ``base_dn``, spherical cells inside,
    smoothed noise inside, clipped.  Semi-axes are (ax, ay, az) micrometres."""
    ax, ay, az = semi_axes
    zc = g.steps * g.dz / 2
    xs = lateral_coords(g.nx, g.dx).astype(np.float32)
    ys = lateral_coords(g.ny, g.dx).astype(np.float32)
    zs = axial_coords(g.steps, g.dz).astype(np.float32)
    dn = np.empty((g.steps, g.ny, g.nx), dtype=np.float32)
    rxy = (xs[None, :] / ax) ** 2 + (ys[:, None] / ay) ** 2
    for k in range(g.steps):
        inside = (rxy + ((zs[k] - zc) / az) ** 2) <= 1.0
        dn[k] = np.where(inside, np.float32(base_dn), np.float32(0))
    # cells: centres uniform inside the ellipsoid (rejection sampling)
    centres = []
    while len(centres) < n_cells:
        p = gen.uniform(-1, 1, (4 * n_cells, 3))
        p = p[(p ** 2).sum(1) <= 1.0]
        centres.extend(p.tolist())
    centres = np.asarray(centres[:n_cells])
    cx, cy, cz = centres[:, 0] * ax, centres[:, 1] * ay, centres[:, 2] * az + zc
    r = gen.uniform(cell_r[0], cell_r[1], n_cells)
    v = gen.uniform(cell_dn[0], cell_dn[1], n_cells)
    add_spheres(dn, g.dx, g.dz, zip(cz, cy, cx), r, v)
    if noise_std > 0:
        sig = noise_sigma_um / g.dx
        coarse = 4 if g.nx * g.ny * g.steps > 64 ** 3 else 1
        noise = smoothed_noise(dn.shape, sig, noise_std, gen, coarse=coarse)
        for k in range(g.steps):
            inside = (rxy + ((zs[k] - zc) / az) ** 2) <= 1.0
            dn[k] += np.where(inside, noise[k], np.float32(0))
        del noise
    np.clip(dn, clip[0], clip[1], out=dn)
    return dn


# ---------------------------------------------------------------------------
# source fields

def _spatial_freqs(nx: int, ny: int, dx: float):
    kx = 2 * np.pi * np.fft.fftfreq(nx, d=dx)
    ky = 2 * np.pi * np.fft.fftfreq(ny, d=dx)
    return kx[None, :], ky[:, None]


def point_source_spectrum(nx: int, ny: int, dx: float, wavelength: float, n0: float,
                          na: float, z_d: float) -> np.ndarray:
    """Angular spectrum of a Gaussian-apodized, NA-limited point source.

    U(k) = exp(-(kt / (k0 NA))^2) * [kt <= k0 NA] * exp(-i kz z_d): a
    converging wave that focuses a distance ``z_d`` after the input plane.
    Natural (unshifted) DFT order, centred on pixel (0, 0).
    """
    k0 = 2 * np.pi / wavelength
    k = n0 * k0
    kx, ky = _spatial_freqs(nx, ny, dx)
    kt2 = kx ** 2 + ky ** 2
    kmax = k0 * na
    pupil = kt2 <= kmax ** 2
    kz = np.sqrt(np.maximum(k * k - kt2, 0.0))
    return np.where(pupil, np.exp(-kt2 / kmax ** 2) * np.exp(-1j * kz * z_d), 0.0)


def point_source_field(nx: int, ny: int, dx: float, wavelength: float, n0: float,
                       na: float, z_d: float, centre=None) -> np.ndarray:
    """complex64 field of one point source, focus ``z_d`` downstream, ||u||_2 = 1.

    ``centre`` is the pixel (iy, ix) of the focus; default the grid centre."""
    u = np.fft.ifft2(point_source_spectrum(nx, ny, dx, wavelength, n0, na, z_d))
    if centre is None:
        centre = (ny // 2, nx // 2)
    u = np.roll(u, (int(centre[0]), int(centre[1])), axis=(0, 1))
    u /= np.linalg.norm(u)
    return u.astype(np.complex64)


def jittered_grid(nx: int, ny: int, pitch: int, jitter: int, gen: np.random.Generator,
                  count: int | None = None):
    """Pixel positions (iy, ix) on a ``pitch`` grid with integer jitter in
    [-jitter, jitter]; when ``count`` is given, a random subset of that size."""
    gy = np.arange(pitch // 2, ny, pitch)
    gx = np.arange(pitch // 2, nx, pitch)
    py, px = np.meshgrid(gy, gx, indexing="ij")
    pos = np.stack([py.ravel(), px.ravel()], axis=1)
    if jitter:
        pos = pos + gen.integers(-jitter, jitter + 1, pos.shape)
    if count is not None and count < len(pos):
        keep = np.sort(gen.choice(len(pos), count, replace=False))
        pos = pos[keep]
    return pos % np.array([ny, nx])


def multiplexed_field(nx: int, ny: int, dx: float, wavelength: float, n0: float,
                      na: float, z_d: float, positions, phases=None) -> np.ndarray:
    """Sum of unit-modulus-weighted copies of one point source.

    u0 = sum_i exp(i phase_i) * shift(u_src, p_i) with integer circular
    shifts; this is the multiplexed input whose march carries every source's
    PSF at once.  Returned as complex64."""
    src = np.fft.ifft2(point_source_spectrum(nx, ny, dx, wavelength, n0, na, z_d))
    src /= np.linalg.norm(src)
    positions = np.asarray(positions, dtype=np.int64).reshape(-1, 2)
    if phases is None:
        phases = np.zeros(len(positions))
    # a comb of weighted deltas, circularly convolved with the single source
    comb = np.zeros((ny, nx), dtype=np.complex128)
    np.add.at(comb, (positions[:, 0] % ny, positions[:, 1] % nx), np.exp(1j * np.asarray(phases)))
    acc = np.fft.fft2(comb)
    spec = np.fft.fft2(src)
    return np.fft.ifft2(spec * acc).astype(np.complex64)


def light_sheet_field(nx: int, ny: int, dx: float, wavelength: float, n0: float,
                      na: float, z_f: float, thin_axis: str = "x") -> np.ndarray:
    """Cylindrical light sheet: Gaussian-apodized up to k0 NA along the thin
    axis, a single (DC) mode along the wide axis, focus ``z_f`` downstream,
    centred on the thin axis; ||u||_2 = 1."""
    k0 = 2 * np.pi / wavelength
    k = n0 * k0
    kx, ky = _spatial_freqs(nx, ny, dx)
    kmax = k0 * na
    if thin_axis == "x":
        kt = np.broadcast_to(kx, (ny, nx))
        wide = np.broadcast_to(ky == 0, (ny, nx))
        shift = (0, nx // 2)
    else:
        kt = np.broadcast_to(ky, (ny, nx))
        wide = np.broadcast_to(kx == 0, (ny, nx))
        shift = (ny // 2, 0)
    kz = np.sqrt(np.maximum(k * k - kt ** 2, 0.0))
    spec = np.where(wide & (np.abs(kt) <= kmax),
                    np.exp(-(kt / kmax) ** 2) * np.exp(-1j * kz * z_f), 0.0)
    u = np.roll(np.fft.ifft2(spec), shift, axis=(0, 1))
    u /= np.linalg.norm(u)
    return u.astype(np.complex64)


# ---------------------------------------------------------------------------
# fluorophores

def fluorophore_density(g: Geometry, n_nuclei: int, r_range=(1.5, 4.0), n_beads: int = 0,
                        gen: np.random.Generator | None = None) -> np.ndarray:
    """Synthetic fluorophore density float32 [steps][ny][nx]: labelled nuclei
    (uniform density 1 inside spheres of radius r_range, centres anywhere in
    the volume) and ``n_beads`` single-voxel beads of density 4."""
    gen = rng(7, 0) if gen is None else gen
    rho = np.zeros((g.steps, g.ny, g.nx), dtype=np.float32)
    c = np.stack([gen.uniform(0, g.steps * g.dz, n_nuclei),
                  gen.uniform(0, g.ny * g.dx, n_nuclei) - g.ny * g.dx / 2,
                  gen.uniform(0, g.nx * g.dx, n_nuclei) - g.nx * g.dx / 2], axis=1)
    add_spheres(rho, g.dx, g.dz, c, gen.uniform(*r_range, n_nuclei), np.ones(n_nuclei))
    np.minimum(rho, 1.0, out=rho)
    if n_beads:
        idx = (gen.integers(0, g.steps, n_beads), gen.integers(0, g.ny, n_beads),
               gen.integers(0, g.nx, n_beads))
        rho[idx] = 4.0
    return rho


# ---------------------------------------------------------------------------
# Bessel beams and Bessel lattices (alternative light-sheet illuminations)

def _annulus(nx, ny, dx, wavelength, na_outer, na_inner):
    k0 = 2 * np.pi / wavelength
    kx, ky = _spatial_freqs(nx, ny, dx)
    kt2 = kx ** 2 + ky ** 2
    if not 0 <= na_inner < na_outer:
        raise ValueError("need 0 <= na_inner < na_outer")
    return kx, ky, (kt2 >= (k0 * na_inner) ** 2) & (kt2 <= (k0 * na_outer) ** 2)


def bessel_spectrum(nx: int, ny: int, dx: float, wavelength: float, n0: float,
                    na_outer: float, na_inner: float) -> np.ndarray:
    """Angular spectrum of a Bessel beam: a flat annulus k0 na_inner <= kt <=
    k0 na_outer (natural DFT order, centred on pixel (0, 0))."""
    _, _, ring = _annulus(nx, ny, dx, wavelength, na_outer, na_inner)
    return ring.astype(np.complex128)


def lattice_spectrum(nx: int, ny: int, dx: float, wavelength: float, n0: float,
                     na_outer: float, na_inner: float, n_points: int = 6, sigma=0.02,
                     phi0: float = 0.0) -> np.ndarray:
    """Angular spectrum of a Bessel lattice: ``n_points`` plane waves whose
    transverse wavevectors k_m = k0 na_r (cos phi_m, sin phi_m) lie on the
    Bessel ring (na_r = (na_outer + na_inner) / 2, phi_m = phi0 + 2 pi m /
    n_points), each a Gaussian spot exp(-((kx - kx_m) / (k0 sx))^2 - ((ky -
    ky_m) / (k0 sy))^2) with (sx, sy) = sigma (NA units; a scalar for both),
    cut to the annulus.  A small sy and a larger sx bound the lattice along x
    into a sheet."""
    k0 = 2 * np.pi / wavelength
    kx, ky, ring = _annulus(nx, ny, dx, wavelength, na_outer, na_inner)
    sx, sy = (sigma, sigma) if np.isscalar(sigma) else sigma
    kr = k0 * 0.5 * (na_outer + na_inner)
    spec = np.zeros((ny, nx))
    for m in range(n_points):
        ph = phi0 + 2 * np.pi * m / n_points
        spec = spec + np.exp(-((kx - kr * np.cos(ph)) / (k0 * sx)) ** 2
                             - ((ky - kr * np.sin(ph)) / (k0 * sy)) ** 2)
    return np.where(ring, spec, 0.0).astype(np.complex128)


def _centred_unit_field(spec, nx, ny, centre):
    u = np.fft.ifft2(spec)
    if centre is None:
        centre = (ny // 2, nx // 2)
    u = np.roll(u, (int(centre[0]), int(centre[1])), axis=(0, 1))
    return (u / np.linalg.norm(u)).astype(np.complex64)


def bessel_field(nx: int, ny: int, dx: float, wavelength: float, n0: float, na_outer: float,
                 na_inner: float, centre=None) -> np.ndarray:
    """complex64 Bessel beam centred on ``centre`` (default the grid centre),
    ||u||_2 = 1."""
    return _centred_unit_field(bessel_spectrum(nx, ny, dx, wavelength, n0, na_outer, na_inner),
                               nx, ny, centre)


def bessel_lattice_field(nx: int, ny: int, dx: float, wavelength: float, n0: float,
                         na_outer: float, na_inner: float, n_points: int = 6, sigma=0.02,
                         phi0: float = 0.0, centre=None) -> np.ndarray:
    """complex64 Bessel lattice (``lattice_spectrum``), ||u||_2 = 1."""
    spec = lattice_spectrum(nx, ny, dx, wavelength, n0, na_outer, na_inner, n_points, sigma,
                            phi0)
    return _centred_unit_field(spec, nx, ny, centre)


# ---------------------------------------------------------------------------
# Perlin gradient noise (the adaptive-optics phantom)

_GRAD12 = np.array([[1, 1, 0], [-1, 1, 0], [1, -1, 0], [-1, -1, 0], [1, 0, 1], [-1, 0, 1],
                    [1, 0, -1], [-1, 0, -1], [0, 1, 1], [0, -1, 1], [0, 1, -1], [0, -1, -1]],
                   dtype=np.float64)


def perlin_noise(shape, cell_vox: float, gen: np.random.Generator) -> np.ndarray:
    """3-D gradient noise on a [nz][ny][nx] grid (Perlin's improved noise:
    gradients from the 12 cube-edge directions chosen by a hashed permutation
    of the lattice, quintic fade 6t^5 - 15t^4 + 10t^3, trilinear blend),
    lattice spacing `cell_vox` voxels.  Values lie in about [-1, 1]."""
    perm = gen.permutation(256)
    perm = np.concatenate([perm, perm])
    nz, ny, nx = shape
    axes = [np.arange(n, dtype=np.float64) / cell_vox for n in (nz, ny, nx)]
    out = np.empty(shape, dtype=np.float64)
    x = axes[2][None, :]
    xi = np.floor(x).astype(np.int64)
    xf = x - xi
    y = axes[1][:, None]
    yi = np.floor(y).astype(np.int64)
    yf = y - yi
    fade = lambda t: t * t * t * (t * (t * 6 - 15) + 10)
    u, v = fade(xf), fade(yf)

    def grad(h, dx_, dy_, dz_):
        g = _GRAD12[h % 12]
        return g[..., 0] * dx_ + g[..., 1] * dy_ + g[..., 2] * dz_

    for k in range(nz):
        z = axes[0][k]
        zi = int(np.floor(z))
        zf = z - zi
        w = fade(zf)
        acc = []
        for cz in (0, 1):
            for cy in (0, 1):
                for cx in (0, 1):
                    h = perm[(perm[(perm[(xi + cx) & 255] + ((yi + cy) & 255)) & 511]
                              + ((zi + cz) & 255)) & 511]
                    acc.append(grad(h, xf - cx, yf - cy, zf - cz))
        lerp = lambda a, b, t: a + t * (b - a)
        x00 = lerp(acc[0], acc[1], u)
        x10 = lerp(acc[2], acc[3], u)
        x01 = lerp(acc[4], acc[5], u)
        x11 = lerp(acc[6], acc[7], u)
        out[k] = lerp(lerp(x00, x10, v), lerp(x01, x11, v), w)
    return out


def perlin_phantom(g: Geometry, feature_um: float = 3.0, octaves: int = 3,
                   sigma: float = 0.03, gen: np.random.Generator | None = None):
    """Synthetic scattering tissue of Perlin noise: n = n0 + sigma * P, P a sum
    of `octaves` noise octaves (lattice spacing feature_um, halved per octave,
    amplitude halved) shifted to zero mean and scaled to unit standard
    deviation (the adaptive-optics paragraph's tissue n = 1.36 +- 0.03, the
    spread read as a standard deviation, with g.n0 = 1.36).  Returns dn = n - n0
    as float32 [steps][ny][nx]."""
    gen = rng(5, 0) if gen is None else gen
    shape = (g.steps, g.ny, g.nx)
    p = np.zeros(shape)
    for o in range(octaves):
        p += perlin_noise(shape, max(feature_um / g.dx / 2 ** o, 1.0), gen) / 2 ** o
    p -= p.mean()
    p /= p.std()
    return (sigma * p).astype(np.float32)


def ao_workload(nxy: int = 256, steps: int = 80):
    """Adaptive-optics workload: a Perlin-noise tissue (n = 1.36 +- 0.03,
    features ~3 um) of nxy^2 x steps voxels at dx = dz = 0.2 um, lambda =
    0.5 um, background n0 = 1.36 (80 slices = 16 um, about four scattering mean
    free paths); a Gaussian-apodised NA 0.6 pupil focusing at the exit plane
    (z_f = steps dz).  Returns (geometry, dn, pupil amplitude, z_f)."""
    g = Geometry(nxy, nxy, steps, 0.2, 0.2, 0.5, 1.36)
    dn = perlin_phantom(g, gen=rng(5, 0))
    k0 = 2 * np.pi / g.wavelength
    kx, ky = _spatial_freqs(g.nx, g.ny, g.dx)
    kt2 = kx ** 2 + ky ** 2
    kmax = k0 * 0.6
    amp = np.where(kt2 <= kmax ** 2, np.exp(-kt2 / kmax ** 2), 0.0).astype(np.float32)
    return g, dn, amp, g.steps * g.dz


# ---------------------------------------------------------------------------
# workloads

def config0():
    """Plain march: 128^2 x 64, dx = dz = 0.1 um, one point source defocused
    2 um (NA 0.6), 20 spheres of radius 1-3 um and dn in [0, 0.05]."""
    g = Geometry(128, 128, 64, 0.1, 0.1, 0.5, 1.33)
    dn = sphere_phantom(g, 20, (1.0, 3.0), (0.0, 0.05), rng(0, 0))
    u0 = point_source_field(g.nx, g.ny, g.dx, g.wavelength, g.n0, 0.6, 2.0)
    return g, u0, dn


def config1(steps: int | None = None, noise: bool = True):
    """Multiplexed PSFs: 512^2 x 512, dx = dz = 0.2 um, 256 sources on a
    jittered 16 x 16 grid (pitch 32 px, jitter +-3 px), random phases; 2000
    spheres (r 1-4 um, n 1.33-1.38) plus smoothed noise (sigma 1 um, std
    0.005), dn clipped to [0, 0.05].  ``steps`` truncates the volume."""
    g = Geometry(512, 512, 512 if steps is None else steps, 0.2, 0.2, 0.5, 1.33)
    n_sph = 2000 if steps is None else max(1, int(round(2000 * g.steps / 512)))
    dn = sphere_phantom(g, n_sph, (1.0, 4.0), (0.0, 0.05), rng(1, 0))
    if noise:
        dn += smoothed_noise(dn.shape, 1.0 / g.dx, 0.005, rng(1, 1),
                             coarse=4 if dn.size > 64 ** 3 else 1)
    np.clip(dn, 0.0, 0.05, out=dn)
    pos = jittered_grid(g.nx, g.ny, 32, 3, rng(1, 2))
    ph = rng(1, 3).uniform(0, 2 * np.pi, len(pos))
    u0 = multiplexed_field(g.nx, g.ny, g.dx, g.wavelength, g.n0, 0.6, 2.0, pos, ph)
    return g, u0, dn


def config2_detection(steps: int | None = None, nxy: int = 1024):
    """Paper-scale detection march: 1024^2 x 1024, dx = dz = 0.2 um, 1000
    multiplexed NA 0.6 sources (32-px pitch grid minus 24 random sites) with
    random phases through an embryo-like ellipsoid (semi-axes 50, 100, 50 um,
    n 1.33-1.38, ~4000 cells).  ``steps``/``nxy`` shrink it for tests."""
    g = Geometry(nxy, nxy, nxy if steps is None else steps, 0.2, 0.2, 0.5, 1.33)
    scale = (g.nx * g.ny * g.steps) / 1024 ** 3
    dn = ellipsoid_phantom(g, (50.0, 100.0, 50.0), max(1, int(round(4000 * scale))),
                           rng(2, 0))
    n_sites = (g.nx // 32) * (g.ny // 32)
    count = max(1, n_sites - 24) if n_sites > 24 else n_sites
    pos = jittered_grid(g.nx, g.ny, 32, 0, rng(2, 1), count=count)
    ph = rng(2, 2).uniform(0, 2 * np.pi, len(pos))
    u0 = multiplexed_field(g.nx, g.ny, g.dx, g.wavelength, g.n0, 0.6, 2.0, pos, ph)
    return g, u0, dn


def config2_light_sheet(g: Geometry, dn_detection: np.ndarray):
    """Light-sheet march of the paper-scale workload: the illumination axis
    becomes the march axis, so the volume is permuted (z <-> x) and the sheet
    (NA 0.15, thin along the detection axis) focuses at the volume centre."""
    dn_t = np.ascontiguousarray(np.transpose(dn_detection, (2, 1, 0)))
    gl = Geometry(g.steps, g.ny, g.nx, g.dx, g.dx, g.wavelength, g.n0)
    u0 = light_sheet_field(gl.nx, gl.ny, gl.dx, gl.wavelength, gl.n0, 0.15,
                           gl.steps * gl.dz / 2, thin_axis="x")
    return gl, u0, dn_t


def config3(steps: int | None = None, nxy: int = 256):
    """Adjoint workload: 256^2 x 512, dx = dz = 0.2 um, 400 spheres (r 1-4 um,
    n 1.33-1.39).  Returns geometry, dn and the pupil amplitude A(k) (NA 0.6
    Gaussian-apodized) with the focal depth z_f of the point source."""
    g = Geometry(nxy, nxy, 512 if steps is None else steps, 0.2, 0.2, 0.5, 1.33)
    n_sph = max(1, int(round(400 * (g.nx * g.ny * g.steps) / (256 * 256 * 512))))
    dn = sphere_phantom(g, n_sph, (1.0, 4.0), (0.0, 0.06), rng(3, 0))
    k0 = 2 * np.pi / g.wavelength
    kx, ky = _spatial_freqs(g.nx, g.ny, g.dx)
    kt2 = kx ** 2 + ky ** 2
    kmax = k0 * 0.6
    amp = np.where(kt2 <= kmax ** 2, np.exp(-kt2 / kmax ** 2), 0.0)
    z_f = g.steps * g.dz
    return g, dn, amp, z_f


def surrogate_volume(child: int, nxy: int = 1024, nz: int = 64) -> np.ndarray:
    """A 64-slice volume of the PSF surrogate's data set (dx = dz = 0.2 um):
    spheres of radius 1-4 um with dn in [0, 0.05] at the density of the
    512^3 multiplexed-PSF workload (about 1000 per 1024^2 x 64 volume) plus
    noise smoothed to 1 um with std 0.005, clipped to [0, 0.05]
    (n 1.33-1.38).  ``child`` selects an independent volume."""
    g = Geometry(nxy, nxy, nz, 0.2, 0.2)
    n_sph = max(1, int(round(2000 * (nxy * nxy * nz) / 512 ** 3)))
    dn = sphere_phantom(g, n_sph, (1.0, 4.0), (0.0, 0.05), rng(4, 2 * child))
    dn += smoothed_noise(dn.shape, 1.0 / g.dx, 0.005, rng(4, 2 * child + 1),
                         coarse=4 if dn.size > 64 ** 3 else 1)
    np.clip(dn, 0.0, 0.05, out=dn)
    return dn


def batch_job_specs(n_jobs: int = 64, sizes=(256, 512, 1024), steps_range=(128, 1024),
                    budget_bytes: float = 160 * 2 ** 30, seed_child: int = 10):
    """Shapes of the uneven batch: nx, ny drawn from ``sizes``, steps uniform
    in ``steps_range``; resampled until dn + intensity fit ``budget_bytes``."""
    gen = rng(2, seed_child)
    while True:
        nx = gen.choice(sizes, n_jobs)
        ny = gen.choice(sizes, n_jobs)
        st = gen.integers(steps_range[0], steps_range[1] + 1, n_jobs)
        total = float((nx.astype(np.int64) * ny * st * 8).sum())
        if total <= budget_bytes:
            return [(int(a), int(b), int(c)) for a, b, c in zip(nx, ny, st)]
