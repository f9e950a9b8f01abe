"""Pins of the warm-start MLP oracle: central finite differences in FP64 (CPU only)."""
import numpy as np

import oracle


def make(seed=0, n=12, d=7, h1=9, h2=8, k=4):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((n, d))
    W1 = rng.standard_normal((d, h1)) * 0.5
    b1 = rng.standard_normal(h1) * 0.1
    W2 = rng.standard_normal((h1, h2)) * 0.5
    b2 = rng.standard_normal(h2) * 0.1
    W3 = rng.standard_normal((h2, k)) * 0.5
    b3 = rng.standard_normal(k) * 0.1
    T = rng.standard_normal((n, k))
    return U, [W1, b1, W2, b2, W3, b3], T


def loss_of(U, params, T):
    Z, _ = oracle.mlp_forward(U, *params)
    return oracle.mlp_loss(Z, T)


def test_backward_matches_central_differences():
    U, params, T = make()
    Z, cache = oracle.mlp_forward(U, *params)
    grads = oracle.mlp_backward(Z, T, cache, params[0], params[2], params[4])
    h = 1e-6
    for p, g in zip(params, grads):
        num = np.zeros_like(p)
        it = np.nditer(p, flags=["multi_index"])
        for _ in it:
            ix = it.multi_index
            old = p[ix]
            p[ix] = old + h
            lp = loss_of(U, params, T)
            p[ix] = old - h
            lm = loss_of(U, params, T)
            p[ix] = old
            num[ix] = (lp - lm) / (2 * h)
        assert np.linalg.norm(num - g) <= 1e-8 * max(1.0, np.linalg.norm(g)) * 100


def test_features_average_of_self_and_neighbours():
    import scipy.sparse as sp
    Xh = np.array([[1.0, 0], [0, 1.0], [0.6, 0.8]])
    P = sp.csr_matrix(np.array([[0, 0.5, 0.5], [1.0, 0, 0], [0, 0, 1.0]]))
    U = oracle.mlp_features(Xh, P)
    assert np.allclose(U[0], 0.5 * (Xh[0] + 0.5 * Xh[1] + 0.5 * Xh[2]))
    assert np.allclose(U[2], Xh[2])
