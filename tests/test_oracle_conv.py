"""Pins of the surrogate's convolution oracle (direct loops, float64).

* forward = scipy.signal.correlate on the zero-padded input (library routine
  for the special case stride 1), plus bias and ReLU;
* a strided layer equals the stride-1 layer sampled every s-th output;
* backward = central finite differences of <conv(x), dy> (tiny shapes) and
  the adjoint identity <conv(x), dy> = <x, dx(dy)>.
"""
import numpy as np
import pytest
from scipy import signal

import oracle


def ref_conv(x, w, b, pad):
    pd, ph, pw = pad
    xp = np.pad(x, ((0, 0), (0, 0), (pd, pd), (ph, ph), (pw, pw)))
    N, Co = x.shape[0], w.shape[0]
    out = []
    for n in range(N):
        ys = []
        for co in range(Co):
            acc = sum(signal.correlate(xp[n, ci], w[co, ci], mode="valid") for ci in range(x.shape[1]))
            ys.append(acc + (b[co] if b is not None else 0))
        out.append(ys)
    return np.array(out)


@pytest.mark.parametrize("kern,pad", [((3, 3, 3), (1, 1, 1)), ((1, 3, 3), (0, 1, 1)), ((3, 1, 2), (1, 0, 0))])
def test_forward_matches_correlate(kern, pad):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 5, 6, 7))
    w = rng.standard_normal((4, 3) + kern)
    b = rng.standard_normal(4)
    y = oracle.conv3d_forward(x, w, b, stride=(1, 1, 1), pad=pad)
    assert np.abs(y - ref_conv(x, w, b, pad)).max() <= 1e-12
    yr = oracle.conv3d_forward(x, w, b, stride=(1, 1, 1), pad=pad, relu=True)
    assert np.array_equal(yr, np.maximum(y, 0))


@pytest.mark.parametrize("stride", [(2, 1, 1), (2, 2, 2), (1, 2, 3)])
def test_stride_is_subsampling(stride):
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 2, 8, 8, 9))
    w = rng.standard_normal((3, 2, 3, 3, 3))
    full = oracle.conv3d_forward(x, w, stride=(1, 1, 1), pad=(1, 1, 1))
    s = oracle.conv3d_forward(x, w, stride=stride, pad=(1, 1, 1))
    sd, sh, sw = stride
    assert np.abs(s - full[:, :, ::sd, ::sh, ::sw]).max() <= 1e-12


@pytest.mark.parametrize("stride", [(1, 1, 1), (2, 1, 1), (2, 2, 2)])
def test_backward_finite_differences(stride):
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 2, 4, 5, 4))
    w = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    y = oracle.conv3d_forward(x, w, b, stride=stride)
    dy = rng.standard_normal(y.shape)
    dx, dw, db = oracle.conv3d_backward(x, w, dy, stride=stride)

    def L(xx, ww, bb):
        return float((oracle.conv3d_forward(xx, ww, bb, stride=stride) * dy).sum())

    h = 1e-6
    for arr, grad, name in ((x, dx, "x"), (w, dw, "w"), (b, db, "b")):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in arr.shape)
            p, m = arr.copy(), arr.copy()
            p[idx] += h
            m[idx] -= h
            args_p = {"x": (p, w, b), "w": (x, p, b), "b": (x, w, p)}[name]
            args_m = {"x": (m, w, b), "w": (x, m, b), "b": (x, w, m)}[name]
            fd = (L(*args_p) - L(*args_m)) / (2 * h)
            assert abs(grad[idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (name, idx)


def test_adjoint_identity():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 4, 8, 6, 6))
    w = rng.standard_normal((5, 4, 3, 3, 3))
    y = oracle.conv3d_forward(x, w, stride=(2, 1, 1))
    dy = rng.standard_normal(y.shape)
    dx, _, _ = oracle.conv3d_backward(x, w, dy, stride=(2, 1, 1))
    assert abs((y * dy).sum() - (x * dx).sum()) <= 1e-10 * abs((y * dy).sum())
