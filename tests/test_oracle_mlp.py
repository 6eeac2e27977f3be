"""Pins for the oracle's warm-start network (CPU only): analytic gradients
against central finite differences in FP64, packing round trip, and one Adam
step against its textbook form."""

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
