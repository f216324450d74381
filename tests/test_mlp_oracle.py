"""Pins of the float64 network oracle: a hand-worked example and finite differences."""
import numpy as np
import pytest

from oracle import mlp


def test_hand_worked_forward_backward():
    # F = 1, H = 1: W1 = 2, b1 = -1, w2 = 3, b2 = 0.5, x = 1, r = 1.5
    # z = 1, h = 1, y = 3.5, e = 2, L = 4, dL/dy = 4,
    # dw2 = 4 h = 4, db2 = 4, dz = 4 w2 = 12, dW1 = 12 x = 12, db1 = 12.
    p = np.array([2.0, -1.0, 3.0, 0.5])
    loss, g = mlp.loss_and_grad(p, [[1.0]], [1.5], H=1)
    assert loss == pytest.approx(4.0)
    assert g.tolist() == pytest.approx([12.0, 12.0, 4.0, 4.0])
    # x = 0: z = -1 is clipped, so only b2 sees a gradient.
    loss, g = mlp.loss_and_grad(p, [[0.0]], [0.0], H=1)
    assert loss == pytest.approx(0.25)
    assert g.tolist() == pytest.approx([0.0, 0.0, 0.0, 1.0])


@pytest.mark.parametrize("F,H", [(1, 32), (2, 32), (3, 8)])
def test_gradient_matches_central_differences(F, H):
    g = np.random.default_rng(F * 100 + H)
    K = 64
    X = g.normal(size=(K, F))
    r = g.normal(size=K)
    p = g.normal(size=mlp.n_params(F, H)) * 0.7
    _, grad = mlp.loss_and_grad(p, X, r, H)
    eps = 1e-6
    num = np.empty_like(p)
    for i in range(len(p)):
        dp = np.zeros_like(p)
        dp[i] = eps
        lp, _ = mlp.loss_and_grad(p + dp, X, r, H)
        lm, _ = mlp.loss_and_grad(p - dp, X, r, H)
        num[i] = (lp - lm) / (2 * eps)
    scale = np.maximum(1.0, np.abs(num))
    assert np.max(np.abs(num - grad) / scale) < 1e-6


def test_forward_matches_loss_path():
    g = np.random.default_rng(0)
    X = g.normal(size=(10, 2))
    p = g.normal(size=mlp.n_params(2, 4))
    y = mlp.forward(p, X, 4)
    loss, _ = mlp.loss_and_grad(p, X, y, 4)
    assert loss == 0.0


def test_adam_first_step_is_signed_lr():
    """At t = 1 the bias-corrected step is lr * g / (|g| + eps)."""
    p = np.array([1.0, -2.0, 0.5])
    grad = np.array([0.3, -4.0, 0.0])
    new, m, v = mlp.adam_step(p, grad, np.zeros(3), np.zeros(3), t=1, lr=0.01)
    assert new.tolist() == pytest.approx([0.99, -1.99, 0.5], abs=1e-9)
    assert m.tolist() == pytest.approx((0.1 * grad).tolist())
    assert v.tolist() == pytest.approx((0.001 * grad * grad).tolist())
