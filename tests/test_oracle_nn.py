"""Pins of the surrogate's FP64 oracle operations (oracle/nn_ref.py) against
closed forms and adjoint identities."""
import numpy as np
import pytest

from oracle import nn_ref


def test_delta_kernel_is_a_periodic_shift():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((2, 4, 5, 6))
    for t, (dz, dy, dx) in enumerate(nn_ref.offsets()):
        W = np.zeros((2, 2, 27))
        W[0, 0, t] = W[1, 1, t] = 1.0
        Y = nn_ref.conv(X, W)
        z, y, x = 1, 2, 3
        assert Y[1, z, y, x] == X[1, (z + dz) % 4, (y + dy) % 5, (x + dx) % 6]


def test_constant_field_gives_the_weight_sum():
    W = np.random.default_rng(1).standard_normal((3, 2, 27))
    X = np.full((2, 4, 4, 4), 2.0)
    Y = nn_ref.conv(X, W, b=np.array([1.0, 0.0, -1.0]))
    assert np.allclose(Y[:, 0, 0, 0], 2.0 * W.sum(axis=(1, 2)) + np.array([1.0, 0.0, -1.0]))


def test_conv_gradients_are_adjoints():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((3, 4, 6, 5))
    W = rng.standard_normal((2, 3, 27))
    G = rng.standard_normal((2, 4, 6, 5))
    lhs = (nn_ref.conv(X, W) * G).sum()
    assert lhs == pytest.approx((X * nn_ref.dgrad(W, G)).sum(), rel=1e-12)
    assert lhs == pytest.approx((W * nn_ref.wgrad(X, G)).sum(), rel=1e-12)


def test_pool_and_up_are_scaled_adjoints():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((2, 4, 6, 8))
    Y = rng.standard_normal((2, 2, 3, 4))
    assert (nn_ref.pool(X) * Y).sum() == pytest.approx((X * nn_ref.up(Y)).sum() / 8, rel=1e-12)
    assert nn_ref.pool(nn_ref.up(Y)) == pytest.approx(Y)


def test_mse_gradient_by_difference():
    rng = np.random.default_rng(4)
    Y, T = rng.standard_normal((3, 2, 3, 4)), rng.standard_normal((3, 2, 3, 4))
    mask = (rng.uniform(size=(2, 3, 4)) > 0.3).astype(float)
    L, dY = nn_ref.mse(Y, T, mask)
    E = np.zeros_like(Y)
    E[1, 1, 2, 3] = 1e-6
    fd = (nn_ref.mse(Y + E, T, mask)[0] - nn_ref.mse(Y - E, T, mask)[0]) / 2e-6
    assert fd == pytest.approx(dY[1, 1, 2, 3], rel=1e-6)


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([3.0, -0.5, 1e-3])
    p, m, v = nn_ref.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), t=1, lr=0.1, eps=0.0)
    assert np.allclose(p, -0.1 * np.sign(g))
