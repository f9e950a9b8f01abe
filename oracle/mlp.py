"""FP64 oracle of the learned warm start (TEST INFRASTRUCTURE ONLY).

The paper has no learned component.  This follows the warm-start design of this
project: a three-layer perceptron d -> h1 -> h2 -> k applied to the one-hop
aggregated, row-normalised attributes U = (X^ + P_N X^) / 2, trained with the
mean squared error against target blocks built from the plain method's own
eigenblocks.  Plain numpy FP64; the backward pass is the analytic chain rule.

Precision model.  The network's products take BF16 operands with wide
accumulation: the input U, the weights and the hidden activations are rounded
to BF16 (FP32 value, then round-to-nearest-even to 8 significant bits), biases
stay FP32.  Passing ``rnd=round_bf16`` reproduces these rounding points in
FP64 arithmetic; ``rnd=None`` is the exact real-valued network.

Parity status:
  mlp_features             pinned (hand-computed walk average)
  mlp_forward/backward     pinned (central finite differences; rounded mode
                           equals exact mode on BF16-representable data)
  round_bf16               pinned (library BF16 conversion)
  adam_step                pinned (closed forms of the first step and of a
                           constant gradient)
  rotated_block, centre_map,
  warm_target              pinned (planted rotation and centre permutation)
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import linear_sum_assignment

__all__ = ["mlp_features", "mlp_forward", "mlp_loss", "mlp_backward", "round_bf16", "adam_step",
           "rotated_block", "centre_map", "warm_target"]


def round_bf16(x):
    """Value of x after FP32 rounding then round-to-nearest-even to BF16 (8 significant
    bits, FP32 exponent range).  Returns float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _ident(a):
    return np.asarray(a, dtype=np.float64)


def mlp_features(Xh, P_N):
    """U = (X^ + P_N X^) / 2: each node's normalised attributes averaged with the mean of
    its topology walk neighbours' (one hop of the walk of Sec. 6.1)."""
    Xh = np.asarray(Xh, dtype=np.float64)
    return 0.5 * (Xh + P_N @ Xh)


def mlp_forward(U, W1, b1, W2, b2, W3, b3, rnd=None):
    """Z^ = relu(relu(U W1 + b1) W2 + b2) W3 + b3, weights laid out (in, out).

    With rnd, U, the weights and both hidden activations pass through rnd before they
    enter a product.  Returns (Z^, cache) where cache holds the product inputs."""
    r = rnd or _ident
    U0 = r(U)
    H1 = r(np.maximum(U0 @ r(W1) + b1, 0.0))
    H2 = r(np.maximum(H1 @ r(W2) + b2, 0.0))
    Z = H2 @ r(W3) + b3
    return Z, (U0, H1, H2)


def mlp_loss(Z, T):
    """L = (1/n) sum_i ||Z_i - T_i||^2 (mean over rows of the squared error)."""
    D = np.asarray(Z, np.float64) - T
    return float((D * D).sum() / Z.shape[0])


def mlp_backward(Z, T, cache, W1, W2, W3, rnd=None):
    """Gradients of mlp_loss with respect to (W1, b1, W2, b2, W3, b3).

    The relu derivative is taken where the stored activation is positive.  With rnd, the
    output gradient and both hidden-layer gradients pass through rnd before they enter a
    product (the same rounding points as the forward pass)."""
    r = rnd or _ident
    U0, H1, H2 = cache
    n = Z.shape[0]
    G3 = r(2.0 * (np.asarray(Z, np.float64) - T) / n)
    dW3 = H2.T @ G3
    db3 = G3.sum(axis=0)
    G2 = r((G3 @ r(W3).T) * (H2 > 0))
    dW2 = H1.T @ G2
    db2 = G2.sum(axis=0)
    G1 = r((G2 @ r(W2).T) * (H1 > 0))
    dW1 = U0.T @ G1
    db1 = G1.sum(axis=0)
    return dW1, db1, dW2, db2, dW3, db3


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One step of Adam (Kingma and Ba, 2015, Algorithm 1) at step count t >= 1: moment
    updates, bias correction by 1 - beta^t, then p - lr m^ / (sqrt(v^) + eps).
    Returns (p, m, v)."""
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return np.asarray(p, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def rotated_block(Q, R):
    """Y = Q~ R: the rows of the n x k block Q scaled to unit L2 norm (zero rows stay zero),
    rotated by the k x k R of a Discretize (Alg. 5), so column c is the soft indicator of
    cluster c."""
    B = np.asarray(Q, np.float64)
    nr = np.sqrt((B * B).sum(axis=1))
    Qt = np.divide(B, nr[:, None], out=np.zeros_like(B), where=nr[:, None] > 0)
    return Qt @ np.asarray(R, np.float64)


def centre_map(labels, Xh, centres):
    """colmap[c] = the centre assigned to cluster c: the assignment (Hungarian method) that
    maximises the total cosine between the clusters' mean attribute vectors and the centres.
    An empty cluster has cosine 0 with every centre."""
    C = np.asarray(centres, np.float64)
    k = C.shape[0]
    C = C / np.linalg.norm(C, axis=1, keepdims=True)
    cos = np.zeros((k, k))
    for c in range(k):
        rows = np.flatnonzero(labels == c)
        if rows.size == 0:
            continue
        mu = np.asarray(Xh, np.float64)[rows].mean(axis=0)
        nm = np.linalg.norm(mu)
        if nm > 0:
            cos[c] = C @ (mu / nm)
    _, colmap = linear_sum_assignment(-cos)
    return colmap


def warm_target(Q, R, labels, Xh, centres):
    """Training target of the warm start from one run of the plain method.

    Q: n x (k+1) orthonormal block of the orthogonal iteration; R: k x k rotation of its
    last Discretize (Alg. 5); labels: that Discretize's labels; Xh: row-normalised
    attributes; centres: the k mixture centres shared by every graph of the family.
    The block Q[:, 1:] is row-normalised and rotated (rotated_block); column c is then moved
    to the centre that cluster c matches (centre_map).
    Returns (T, colmap) with T[:, colmap[c]] = Y[:, c]."""
    k = R.shape[0]
    Y = rotated_block(np.asarray(Q, np.float64)[:, 1:k + 1], R)
    colmap = centre_map(labels, Xh, centres)
    T = np.zeros_like(Y)
    T[:, colmap] = Y
    return T, colmap
