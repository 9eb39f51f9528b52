"""Pins of the camera-image oracle (oracle/image.py).

* the hat weights of the PSF nodes sum to one at every pixel;
* identical node PSFs give the periodic convolution of the emission with that
  PSF (computed by FFT);
* one emitter on a node gives that node's PSF at its position, also across
  the image edge;
* an emitter a quarter of the pitch from a node gives 3/4 and 1/4 of the two
  nodes' PSFs;
* the image integrates to sum(E) for PSFs of unit sum.
"""
import numpy as np

from oracle import image as oim


def test_hat_weights_partition_unity():
    for n, p in ((64, 16), (128, 32), (96, 32)):
        w = oim.hat_weights(n, p)
        assert np.abs(w.sum(axis=0) - 1).max() <= 1e-15


def test_invariant_psf_is_a_convolution():
    rng = np.random.default_rng(0)
    E = rng.uniform(0, 1, (64, 96))
    psf = rng.uniform(0, 1, (16, 16))
    P = np.broadcast_to(psf, (4, 6, 16, 16))
    got = oim.accumulate(np.zeros((64, 96)), E, P, 16)
    ref = oim.accumulate_fft(np.zeros((64, 96)), E, psf)
    assert np.abs(got - ref).max() <= 1e-12 * ref.max()


def test_emitter_on_a_node_and_between_nodes():
    rng = np.random.default_rng(1)
    P = rng.uniform(0, 1, (4, 4, 8, 8))
    E = np.zeros((64, 64))
    E[8, 56] = 2.0                      # node (0, 3); its crop wraps over the left edge
    got = oim.accumulate(np.zeros((64, 64)), E, P, 16)
    ref = np.zeros((64, 64))
    ref[np.ix_((8 - 4 + np.arange(8)) % 64, (56 - 4 + np.arange(8)) % 64)] = 2.0 * P[0, 3]
    assert np.abs(got - ref).max() <= 1e-15
    E = np.zeros((64, 64))
    E[24, 28] = 1.0                     # 1/4 pitch right of node (1, 1) = (24, 24)
    got = oim.accumulate(np.zeros((64, 64)), E, P, 16)
    ref = np.zeros((64, 64))
    ref[np.ix_(24 - 4 + np.arange(8), 28 - 4 + np.arange(8))] = 0.75 * P[1, 1] + 0.25 * P[1, 2]
    assert np.abs(got - ref).max() <= 1e-15


def test_image_integrates_to_the_emission():
    rng = np.random.default_rng(2)
    P = rng.uniform(0, 1, (2, 2, 16, 16))
    P /= P.sum(axis=(2, 3), keepdims=True)
    E = rng.uniform(0, 1, (64, 64))
    got = oim.accumulate(np.zeros((64, 64)), E, P, 32)
    assert abs(got.sum() - E.sum()) <= 1e-10 * E.sum()
