"""Float64 oracle of the split-predictor network: TEST INFRASTRUCTURE ONLY.

The paper has no learned component; this network is the project's own
addition on top of the exact split search (Theorem 14).  The oracle states the
network in its plainest form so that the GPU forward/backward/optimiser
kernels can be checked against it:

    z = W1 x + b1          (W1: H x F, b1: H)
    h = relu(z)            (relu'(z) taken as 1 for z > 0, else 0)
    y = w2 . h + b2        (w2: H, b2: scalar)
    L = mean_k (y_k - r_k)^2

Parameter vector layout: [W1 row-major (H*F), b1 (H), w2 (H), b2 (1)].
Adam: m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
      p <- p - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np


def n_params(F: int, H: int) -> int:
    return H * F + 2 * H + 1


def unpack(params: np.ndarray, F: int, H: int):
    p = np.asarray(params, dtype=np.float64)
    W1 = p[: H * F].reshape(H, F)
    b1 = p[H * F: H * F + H]
    w2 = p[H * F + H: H * F + 2 * H]
    b2 = p[H * F + 2 * H]
    return W1, b1, w2, b2


def forward(params, X, H: int) -> np.ndarray:
    X = np.asarray(X, dtype=np.float64)
    W1, b1, w2, b2 = unpack(params, X.shape[1], H)
    h = np.maximum(X @ W1.T + b1, 0.0)
    return h @ w2 + b2


def loss_and_grad(params, X, r, H: int):
    """Mean-squared-error loss and its exact gradient (chain rule, by hand)."""
    X = np.asarray(X, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    K, F = X.shape
    W1, b1, w2, b2 = unpack(params, F, H)
    z = X @ W1.T + b1
    h = np.maximum(z, 0.0)
    y = h @ w2 + b2
    e = y - r
    loss = float(np.mean(e * e))
    gy = 2.0 * e / K                      # dL/dy_k
    g_w2 = h.T @ gy
    g_b2 = gy.sum()
    gz = np.outer(gy, w2) * (z > 0.0)     # dL/dz_kj
    g_W1 = gz.T @ X
    g_b1 = gz.sum(axis=0)
    grad = np.concatenate([g_W1.ravel(), g_b1, g_w2, [g_b2]])
    return loss, grad


def adam_step(params, grad, m, v, t: int, lr: float, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8):
    p = np.asarray(params, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
