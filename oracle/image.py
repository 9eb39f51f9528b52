"""FP64 oracle of the camera image (Fig. 1c; main-text paragraph on the
light-sheet simulation: convolving the spatially varying PSFs with the
fluorescent object gives the image seen by the camera).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``.

Fluorescence is incoherent, so the camera image adds intensities: an emitter
at x' of depth z with emission E(x', z) = excitation(x', z) * density(x', z)
contributes E(x', z) * PSF_{x', z}(x - x') to the camera pixel x, where
PSF_{x', z} is the detection PSF of a point at (x', z) in the plane the
camera is focused on.  The PSFs are known on a grid of nodes g (pitch P,
node g at pixel (P/2 + P i, P/2 + P j)) from multiplexed marches; between
nodes they are blended with the bilinear hat weights
phi_g(x') = h((x'_y - g_y) / P) h((x'_x - g_x) / P), h(t) = max(0, 1 - |t|),
measured periodically (a partition of unity), so that

    image(x) += sum_{x'} E(x', z) sum_g phi_g(x') PSF_g(x - x')

for each depth slab z, with PSF_g a C x C crop whose centre (C/2, C/2) is the
emitter and periodic image indices.

Parity status (tests/test_oracle_image.py): identical node PSFs give the
periodic convolution of E with that PSF (FFT, independent); an emitter on a
node gives that node's PSF; an emitter between two nodes gives the hat-weighted
blend; the image integrates to sum E * sum PSF for unit-sum PSFs.
"""
from __future__ import annotations

import numpy as np


def hat_weights(n: int, pitch: int):
    """[n_nodes][n] periodic bilinear weights of nodes at pitch/2 + pitch i."""
    nodes = pitch // 2 + pitch * np.arange(n // pitch)
    x = np.arange(n)
    d = (x[None, :] - nodes[:, None] + n // 2) % n - n // 2
    return np.maximum(0.0, 1.0 - np.abs(d) / pitch)


def accumulate(image, emission, node_psfs, pitch):
    """image [ny][nx] += the camera image of one emission slab [ny][nx] with
    node PSFs [gy][gx][C][C] (returns the new image, float64)."""
    E = np.asarray(emission, float)
    ny, nx = E.shape
    P = np.asarray(node_psfs, float)
    gy, gx, C, _ = P.shape
    wy, wx = hat_weights(ny, pitch), hat_weights(nx, pitch)
    out = np.array(image, float, copy=True)
    for i in range(gy):
        for j in range(gx):
            src = E * np.outer(wy[i], wx[j])            # the part of E that uses node (i, j)
            ys, xs = np.nonzero(src)
            for y, x in zip(ys, xs):
                rows = (y - C // 2 + np.arange(C)) % ny
                cols = (x - C // 2 + np.arange(C)) % nx
                out[np.ix_(rows, cols)] += src[y, x] * P[i, j]
    return out


def accumulate_fft(image, emission, psf):
    """The same for one spatially invariant PSF: a periodic convolution."""
    E = np.asarray(emission, float)
    ny, nx = E.shape
    C = np.shape(psf)[0]
    k = np.zeros((ny, nx))
    rows = (np.arange(C) - C // 2) % ny
    cols = (np.arange(C) - C // 2) % nx
    k[np.ix_(rows, cols)] = psf
    return np.asarray(image, float) + np.real(np.fft.ifft2(np.fft.fft2(E) * np.fft.fft2(k)))
