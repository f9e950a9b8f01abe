"""FP64 oracle of the learned warm start (TEST INFRASTRUCTURE ONLY).

The paper has no learned component; this follows the warm-start design of this
project: a three-layer perceptron d -> h1 -> h2 -> k applied to the one-hop
aggregated, row-normalised attributes U = (X^ + P_N X^) / 2, trained with the
mean squared error against target blocks.  Plain numpy FP64; the backward pass
is the analytic chain rule.
"""
from __future__ import annotations

import numpy as np

__all__ = ["mlp_features", "mlp_forward", "mlp_loss", "mlp_backward"]


def mlp_features(Xh, P_N):
    """U = (X^ + P_N X^) / 2: each node's normalised attributes averaged with the mean of
    its topology walk neighbours' (one hop of the walk of Sec. 6.1)."""
    Xh = np.asarray(Xh, dtype=np.float64)
    return 0.5 * (Xh + P_N @ Xh)


def mlp_forward(U, W1, b1, W2, b2, W3, b3):
    """Z^ = relu(relu(U W1 + b1) W2 + b2) W3 + b3; returns (Z^, cache)."""
    A1 = np.asarray(U, np.float64) @ W1 + b1
    H1 = np.maximum(A1, 0.0)
    A2 = H1 @ W2 + b2
    H2 = np.maximum(A2, 0.0)
    Z = H2 @ W3 + b3
    return Z, (np.asarray(U, np.float64), A1, H1, A2, H2)


def mlp_loss(Z, T):
    """L = (1/n) sum_i ||Z_i - T_i||^2 (mean over rows of the squared error)."""
    D = np.asarray(Z, np.float64) - T
    return float((D * D).sum() / Z.shape[0])


def mlp_backward(Z, T, cache, W1, W2, W3):
    """Gradients of mlp_loss with respect to (W1, b1, W2, b2, W3, b3)."""
    U, A1, H1, A2, H2 = cache
    n = Z.shape[0]
    dZ = 2.0 * (np.asarray(Z, np.float64) - T) / n
    dW3 = H2.T @ dZ
    db3 = dZ.sum(axis=0)
    dA2 = (dZ @ W3.T) * (A2 > 0)
    dW2 = H1.T @ dA2
    db2 = dA2.sum(axis=0)
    dA1 = (dA2 @ W2.T) * (A1 > 0)
    dW1 = U.T @ dA1
    db1 = dA1.sum(axis=0)
    return dW1, db1, dW2, db2, dW3, db3
