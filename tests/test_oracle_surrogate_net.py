"""Pins of the surrogate network's FP64 reference (oracle/surrogate_net.py).

* the bfloat16 rounding equals torch's float32 -> bfloat16 conversion;
* the float64 loss gradient (rnd=False) matches central finite differences
  on coordinates of every layer and of the error head;
* a target equal to the network's own PSF gives zero PSF-term gradient, and
  lam = 0 gives a zero error-head gradient.
"""
import numpy as np
import pytest
import torch

from oracle import surrogate_net as net


def random_params(rng, scale=1.0):
    p = {"w": [], "b": []}
    for Ci, Co, k, _, _ in net.LAYERS:
        fan = Ci * k[0] * k[1] * k[2]
        p["w"].append(rng.standard_normal((Co, Ci) + k) * np.sqrt(2.0 / fan) * scale)
        p["b"].append(rng.standard_normal(Co) * 0.1)
    p["b"][5] = p["b"][5] - 2.0
    p["we"] = rng.standard_normal(net.HEAD_C) * 0.5
    p["be"] = -1.0
    return p


def sample(rng, B=1):
    dn = rng.uniform(0, 0.05, (B, 64, 32, 32))
    depth = rng.integers(0, 64, B).astype(np.float64)
    target = rng.uniform(0, 1, (B, 32, 32, 32))
    return dn, depth, target


def test_bf16_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-8, 8, 10000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.5]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(net.bf16(x), ref)


def total_loss(p, dn, depth, target, lam, r_fixed):
    c = net.forward(p, dn, depth, rnd=False)
    a, b, _ = net.loss(c, target, lam, r_fixed)
    return a + b


def test_gradient_finite_differences():
    rng = np.random.default_rng(1)
    p = random_params(rng)
    dn, depth, target = sample(rng)
    lam = 0.7
    c = net.forward(p, dn, depth, rnd=False)
    g = net.backward(p, c, target, lam, rnd=False)
    r0 = net.loss(c, target, lam)[2]   # the head's target error is held constant
    checks = [("w", l) for l in range(6)] + [("b", 0), ("b", 5), ("we", None), ("be", None)]
    for kind, l in checks:
        arr = p[kind][l] if l is not None else p[kind]
        grad = g[kind][l] if l is not None else g[kind]
        if np.ndim(arr) == 0:
            idx = ()
        else:
            # a coordinate with a gradient well above the noise floor
            flat = np.argsort(np.abs(np.asarray(grad)).ravel())[-5:]
            idx = np.unravel_index(flat[rng.integers(0, 5)], np.shape(arr))
        h = 1e-7 * max(1.0, abs(float(np.asarray(arr)[idx])))

        def at(delta):
            q = {"w": list(p["w"]), "b": list(p["b"]), "we": p["we"], "be": p["be"]}
            if l is None:
                v = np.array(p[kind], dtype=np.float64, copy=True)
                v[idx] += delta
                q[kind] = v if np.ndim(v) else float(v)
            else:
                v = p[kind][l].copy()
                v[idx] += delta
                q[kind][l] = v
            return total_loss(q, dn, depth, target, lam, r0)

        fd = (at(h) - at(-h)) / (2 * h)
        gv = float(np.asarray(grad)[idx])
        assert abs(gv - fd) <= 1e-5 * max(abs(fd), 1e-8), (kind, l, gv, fd)


def test_fixed_points():
    rng = np.random.default_rng(2)
    p = random_params(rng)
    dn, depth, _ = sample(rng, B=2)
    c = net.forward(p, dn, depth, rnd=False)
    g = net.backward(p, c, c["psf"] + 1e-300, lam=0.0, rnd=False)
    for l in range(6):
        assert np.abs(g["w"][l]).max() <= 1e-12 and np.abs(g["b"][l]).max() <= 1e-12
    assert np.abs(g["we"]).max() == 0.0 and g["be"] == 0.0
