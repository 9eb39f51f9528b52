"""Pins of the oracle's Adam step (oracle/surrogate_net.py: adam_step).

Each pin fixes a part a plausible slip would break: the first step from zero
moments (bias correction at t = 1), constant gradients (bias correction at
every t; swapped betas fail), the unrolled sums of the two moment recursions
over a random gradient sequence, and descent on a quadratic (the sign).
"""
import numpy as np
import pytest

from oracle import surrogate_net as net


def test_first_step_from_zero_moments():
    """m_hat = g and v_hat = g^2 after one step, so dw = -lr g / (|g| + eps)."""
    rng = np.random.default_rng(0)
    g = rng.standard_normal(1000) * np.logspace(-9, 2, 1000)
    lr, eps = 1e-3, 1e-8
    w1, m1, v1 = net.adam_step(np.zeros_like(g), g, np.zeros_like(g), np.zeros_like(g), 1, lr,
                               eps=eps)
    assert np.allclose(w1, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
    assert np.allclose(m1, 0.1 * g, rtol=1e-15) and np.allclose(v1, 0.001 * g * g, rtol=1e-15)


@pytest.mark.parametrize("beta1,beta2", [(0.9, 0.999), (0.5, 0.9)])
def test_constant_gradient_gives_unit_steps(beta1, beta2):
    """With g constant the bias-corrected moments are exactly g and g^2 at
    every step: each step moves w by -lr g / (|g| + eps)."""
    g = np.array([3.0, -0.25, 1e-3])
    m, v = np.zeros(3), np.zeros(3)
    lr, eps = 0.01, 1e-8
    for t in range(1, 40):
        step, m, v = net.adam_step(np.zeros(3), g, m, v, t, lr, beta1, beta2, eps)
        assert np.allclose(step, -lr * g / (np.abs(g) + eps), rtol=1e-10, atol=0), t


def test_unrolled_moment_sums():
    """m_T = (1 - b1) sum_i b1^(T-i) g_i, v_T = (1 - b2) sum_i b2^(T-i) g_i^2,
    and w_T = w_0 - lr sum_t m_hat_t / (sqrt(v_hat_t) + eps), evaluated from
    the sums directly (not by the recursion) over 25 random gradients."""
    rng = np.random.default_rng(3)
    T, n = 25, 7
    G = rng.standard_normal((T, n))
    b1, b2, lr, eps = 0.9, 0.999, 2e-3, 1e-8
    w0 = rng.standard_normal(n)
    w, m, v = w0.copy(), np.zeros(n), np.zeros(n)
    for t in range(1, T + 1):
        w, m, v = net.adam_step(w, G[t - 1], m, v, t, lr, b1, b2, eps)
    step_sum = np.zeros(n)
    for t in range(1, T + 1):
        mt = (1 - b1) * sum(b1 ** (t - i) * G[i - 1] for i in range(1, t + 1))
        vt = (1 - b2) * sum(b2 ** (t - i) * G[i - 1] ** 2 for i in range(1, t + 1))
        step_sum += (mt / (1 - b1 ** t)) / (np.sqrt(vt / (1 - b2 ** t)) + eps)
    assert np.allclose(m, mt, rtol=1e-13) and np.allclose(v, vt, rtol=1e-13)
    assert np.allclose(w, w0 - lr * step_sum, rtol=1e-12, atol=1e-15)


def test_descends_a_quadratic():
    """f(w) = |w - a|^2 / 2, g = w - a: the iterates approach a."""
    a = np.array([1.5, -2.0, 0.3])
    w, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 3001):
        w, m, v = net.adam_step(w, w - a, m, v, t, 0.01)
    assert np.abs(w - a).max() < 1e-2


def test_step_count_starts_at_one():
    with pytest.raises(ValueError):
        net.adam_step(np.zeros(1), np.ones(1), np.zeros(1), np.zeros(1), 0, 1e-3)
