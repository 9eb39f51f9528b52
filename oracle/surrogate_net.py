"""FP64 reference of the PSF surrogate network: forward, loss and backward.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``).  The surrogate is
this project's own learned component; the paper has none.  The network is
written out here from its definition, in NCDHW float64 with the convolutions
of ``conv3d_forward`` / ``conv3d_backward`` (direct loops):

  x0      5 channels on the [64][32][32] patch, padded with zeros to 8:
          dn * 20, the mask [z >= depth], the lateral coordinates
          cy = (y - 15.5) / 16, cx = (x - 15.5) / 16 and cy^2 + cx^2
  c1..c4  3x3x3 convolutions, 32 channels, pad 1, strides (2,2,2) then (2,1,1)
          three times, ReLU                                   -> [32][4][16][16]
  d1      4x3x3 convolution, 64 channels, pad (0,1,1), ReLU    -> [64][1][16][16]
  up      nearest-neighbour x2 in y and x                      -> [64][1][32][32]
  d2      1x3x3 convolution, 32 channels, pad (0,1,1), softplus -> PSF [32][32][32]
  head    err = softplus(we . mean_{y,x}(d1) + be)
  loss    mean_n r_n^2 + lam mean_n (err_n - r_n)^2,  r_n = |psf_n - t_n| / |t_n|
          (r_n is a constant of the head term: no gradient flows through it)

With ``rnd=True`` every stored activation and every stored gradient map is
rounded to bfloat16 (round to nearest even) at the points where the network
stores them in that format: the input, each ReLU output, the PSF layer's
pre-activation gradient, the gradient at the upsampled map and each masked
gradient handed to the layer below.  Arithmetic stays float64.  With
``rnd=False`` the network is a smooth float64 function (finite-difference
pins).

The optimizer step ``adam_step`` is Adam (Kingma & Ba, "Adam: a method for
stochastic optimization", ICLR 2015, Algorithm 1): exponential moving
averages of the gradient and of its square, each divided by its bias
correction, then w -= lr m_hat / (sqrt(v_hat) + eps).

Parity status: the network is pinned by central finite differences of the
loss in float64 (tests/test_oracle_surrogate_net.py); the convolutions
themselves are pinned in tests/test_oracle_conv.py; ``adam_step`` by the
closed form of the first step from zero moments, by constant gradients
(bias-corrected moments exact at every step), by the unrolled sums of the
moment recursions and by convergence on a quadratic
(tests/test_oracle_adam.py).
"""
from __future__ import annotations

import numpy as np

from . import conv3d_backward, conv3d_forward

# (Ci, Co, kernel, stride, pad) of c1, c2, c3, c4, d1, d2
LAYERS = (
    (8, 32, (3, 3, 3), (2, 2, 2), (1, 1, 1)),
    (32, 32, (3, 3, 3), (2, 1, 1), (1, 1, 1)),
    (32, 32, (3, 3, 3), (2, 1, 1), (1, 1, 1)),
    (32, 32, (3, 3, 3), (2, 1, 1), (1, 1, 1)),
    (32, 64, (4, 3, 3), (1, 1, 1), (0, 1, 1)),
    (64, 32, (1, 3, 3), (1, 1, 1), (0, 1, 1)),
)
HEAD_C = 64


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64.

    The value is first rounded to float32, since the kernels round float32
    results to bfloat16."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def softplus(z):
    return np.where(z > 20.0, z, np.log1p(np.exp(np.minimum(z, 20.0))))


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def prep_input(dn, depth, rnd=True):
    """x0 [B][8][64][32][32] from dn [B][64][32][32] and depth [B] (slices)."""
    dn = np.asarray(dn, dtype=np.float64)
    B, D = dn.shape[0], dn.shape[1]
    x = np.zeros((B, 8) + dn.shape[1:])
    x[:, 0] = dn * 20.0
    z = np.arange(D, dtype=np.float64)
    x[:, 1] = (z[None, :] >= np.asarray(depth, dtype=np.float64)[:, None])[:, :, None, None]
    c = (np.arange(dn.shape[2]) - 15.5) / 16.0
    x[:, 2] = c[None, None, :, None]
    x[:, 3] = c[None, None, None, :]
    x[:, 4] = c[None, None, :, None] ** 2 + c[None, None, None, :] ** 2
    return bf16(x) if rnd else x


def forward(params, dn, depth, rnd=True):
    """params: dict with w[l] [Co][Ci][kd][kh][kw], b[l] [Co], we [64], be ()."""
    x = prep_input(dn, depth, rnd)
    acts = [x]
    a = x
    for l in range(5):
        _, _, _, stride, pad = LAYERS[l]
        a = conv3d_forward(a, params["w"][l], params["b"][l], stride=stride, pad=pad, relu=True)
        if rnd:
            a = bf16(a)
        acts.append(a)
    a5 = acts[5]                                     # [B][64][1][16][16]
    u = a5.repeat(2, axis=3).repeat(2, axis=4)       # [B][64][1][32][32]
    _, _, _, stride, pad = LAYERS[5]
    z6 = conv3d_forward(u, params["w"][5], params["b"][5], stride=stride, pad=pad)[:, :, 0]
    psf = softplus(z6)                               # [B][32][32][32]
    pooled = a5.mean(axis=(2, 3, 4))                 # [B][64]
    epre = pooled @ params["we"] + params["be"]
    err = softplus(epre)
    return {"acts": acts, "u": u, "z6": z6, "psf": psf, "pooled": pooled, "epre": epre,
            "err": err}


def loss(cache, target, lam, r_fixed=None):
    """(psf term, head term, per-sample r) of the batch loss.  ``r_fixed``
    replaces r in the head term (the constant the gradient treats it as)."""
    t = np.asarray(target, dtype=np.float64)
    B = t.shape[0]
    d = (cache["psf"] - t).reshape(B, -1)
    tt = (t.reshape(B, -1) ** 2).sum(axis=1)
    r2 = (d ** 2).sum(axis=1) / tt
    r = np.sqrt(r2)
    rh = r if r_fixed is None else r_fixed
    return r2.mean(), lam * ((cache["err"] - rh) ** 2).mean(), r


def backward(params, cache, target, lam, rnd=True):
    """Gradients of loss() (sum of both terms) with respect to every parameter."""
    t = np.asarray(target, dtype=np.float64)
    B = t.shape[0]
    rb = bf16 if rnd else (lambda v: v)
    tt = (t.reshape(B, -1) ** 2).sum(axis=1)
    _, _, r = loss(cache, t, lam)
    dz6 = rb(2.0 / (B * tt)[:, None, None, None] * (cache["psf"] - t) * sigmoid(cache["z6"]))
    depre = 2.0 * lam * (cache["err"] - r) / B * sigmoid(cache["epre"])
    grads = {"w": [None] * 6, "b": [None] * 6}
    grads["we"] = cache["pooled"].T @ depre
    grads["be"] = depre.sum()
    dpool = depre[:, None] * params["we"][None, :]    # [B][64]
    _, _, _, stride, pad = LAYERS[5]
    du, grads["w"][5], grads["b"][5] = conv3d_backward(cache["u"], params["w"][5],
                                                       dz6[:, :, None], stride=stride, pad=pad)
    du = rb(du)
    a5 = cache["acts"][5]
    Bc, C, _, h, w = a5.shape
    da5 = du.reshape(Bc, C, 1, h, 2, w, 2).sum(axis=(4, 6)) + (dpool / (h * w))[:, :, None, None,
                                                                                  None]
    dz = rb(da5 * (a5 > 0))
    for l in range(4, -1, -1):
        _, _, _, stride, pad = LAYERS[l]
        dx, grads["w"][l], grads["b"][l] = conv3d_backward(cache["acts"][l], params["w"][l], dz,
                                                           stride=stride, pad=pad)
        if l > 0:
            dz = rb(dx * (cache["acts"][l] > 0))
    return grads


def adam_step(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1 (Kingma & Ba 2015, Algorithm 1), float64.

    Returns (w_new, m_new, v_new); inputs are not modified."""
    if t < 1:
        raise ValueError("Adam steps are counted from 1")
    w, g = np.asarray(w, np.float64), np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return w - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
