"""Pins for the oracle's warm-start network (CPU only): analytic gradients
against central finite differences in FP64, packing round trip, Adam's first
step, two Adam steps worked by hand, and Adam under a constant gradient."""

import numpy as np

from oracle import mlp


def test_pack_roundtrip():
    rng = np.random.default_rng(0)
    ni, h, no = 3, 5, 4
    p = rng.standard_normal(mlp.param_count(ni, h, no))
    assert np.array_equal(mlp.pack(mlp.unpack(p, ni, h, no)), p)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    ni, h, no, B = 3, 6, 4, 7
    p = mlp.init_params(rng, ni, h, no) + 0.05 * rng.standard_normal(mlp.param_count(ni, h, no))
    x = rng.standard_normal((B, ni))
    t = rng.standard_normal((B, no))
    L, g = mlp.loss_and_grads(p, x, t, ni, h, no)
    num = np.empty_like(p)
    eps = 1e-6
    for k in range(p.size):
        e = np.zeros_like(p)
        e[k] = eps
        num[k] = (mlp.loss_and_grads(p + e, x, t, ni, h, no)[0]
                  - mlp.loss_and_grads(p - e, x, t, ni, h, no)[0]) / (2 * eps)
    np.testing.assert_allclose(g, num, rtol=1e-5, atol=1e-8)
    assert L > 0


def test_forward_is_relu_mlp():
    rng = np.random.default_rng(2)
    ni, h, no = 2, 3, 2
    p = rng.standard_normal(mlp.param_count(ni, h, no))
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p, ni, h, no)
    x = rng.standard_normal((4, ni))
    y, _ = mlp.forward(p, x, ni, h, no)
    for r in range(4):
        a = np.maximum(W1 @ x[r] + b1, 0)
        a = np.maximum(W2 @ a + b2, 0)
        np.testing.assert_allclose(y[r], W3 @ a + b3, rtol=1e-14)


def test_adam_first_step_moves_by_lr():
    # with m = v = 0, the first bias-corrected Adam step is -lr * sign(g)
    # (up to eps)
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(p, -0.01 * np.sign(g), rtol=1e-4)


def test_adam_two_steps_worked_by_hand():
    # p0 = 1, gradients 0.5 then -0.25, lr 0.1 (beta1 0.9, beta2 0.999,
    # eps 1e-8), worked in 40-digit decimal arithmetic:
    #   step 1: m = 0.05, v = 0.00025, m_hat = 0.5, v_hat = 0.25,
    #           p = 1 - 0.1 * 0.5 / (0.5 + 1e-8) = 0.90000000199999996...
    #   step 2: m = 0.02, v = 0.00031225, m_hat = 0.02 / 0.19,
    #           v_hat = 0.00031225 / 0.001999, p = 0.87336629870784616...
    p, m, v = np.array([1.0]), np.zeros(1), np.zeros(1)
    p, m, v = mlp.adam_step(p, np.array([0.5]), m, v, 1, lr=0.1)
    np.testing.assert_allclose([m[0], v[0], p[0]], [0.05, 0.00025, 0.90000000199999996], rtol=1e-15)
    p, m, v = mlp.adam_step(p, np.array([-0.25]), m, v, 2, lr=0.1)
    np.testing.assert_allclose([m[0], v[0]], [0.02, 0.00031225], rtol=1e-14)
    np.testing.assert_allclose(p[0], 0.87336629870784616256, rtol=1e-15)


def test_adam_constant_gradient_steps():
    # with a constant gradient g the bias-corrected moments are exactly g and
    # g^2 at every step, so each step moves by lr |g| / (|g| + eps) against
    # the sign of g
    g = np.array([2.0, -0.003, 0.7])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for step in range(1, 26):
        p, m, v = mlp.adam_step(p, g, m, v, step, lr=0.01)
    np.testing.assert_allclose(p, -25 * 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9)
