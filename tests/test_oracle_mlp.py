"""Pins of the warm-start oracle (CPU only): central finite differences in FP64, the
library BF16 conversion, closed forms of Adam, and a planted rotation for the target."""
import numpy as np
import pytest
import torch

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


def test_relu_mask_and_bias_gradients_by_hand():
    # one row, identity-like weights: the gradient flows only through positive units
    U = np.array([[1.0, -2.0]])
    W1 = np.eye(2)
    b1 = np.zeros(2)
    W2 = np.eye(2)
    b2 = np.zeros(2)
    W3 = np.array([[1.0], [1.0]])
    b3 = np.zeros(1)
    T = np.array([[0.0]])
    Z, cache = oracle.mlp_forward(U, W1, b1, W2, b2, W3, b3)
    assert Z[0, 0] == 1.0                      # relu drops the -2
    dW1, db1, dW2, db2, dW3, db3 = oracle.mlp_backward(Z, T, cache, W1, W2, W3)
    assert db3[0] == 2.0                       # 2 (Z - T) / n
    assert np.array_equal(db2, [2.0, 0.0]) and np.array_equal(db1, [2.0, 0.0])
    assert np.array_equal(dW3[:, 0], [2.0, 0.0])
    assert np.array_equal(dW1, [[2.0, 0.0], [-4.0, 0.0]])


def test_round_bf16_matches_library_conversion():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 1.0 + 2.0 ** -9, 1.0 + 3 * 2.0 ** -9,
                         -1.0 - 2.0 ** -9, 3.0e38, 1.0e-40]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(oracle.round_bf16(x), ref)
    # ties go to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert oracle.round_bf16(1.0 + 2.0 ** -8) == 1.0
    assert oracle.round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2 * 2.0 ** -7


def test_rounded_network_equals_exact_on_representable_values():
    # small integers and their sums are exact in BF16 and FP32: the rounding points
    # leave such a network unchanged, forward and backward
    rng = np.random.default_rng(4)
    U = rng.integers(-3, 4, (6, 5)).astype(float)
    W1 = rng.integers(-2, 3, (5, 4)).astype(float)
    W2 = rng.integers(-2, 3, (4, 3)).astype(float)
    W3 = rng.integers(-2, 3, (3, 2)).astype(float)
    b1, b2, b3 = np.zeros(4), np.ones(3), np.zeros(2)
    T = rng.integers(-3, 4, (6, 2)).astype(float)
    Z0, c0 = oracle.mlp_forward(U, W1, b1, W2, b2, W3, b3)
    Z1, c1 = oracle.mlp_forward(U, W1, b1, W2, b2, W3, b3, rnd=oracle.round_bf16)
    assert np.array_equal(Z0, Z1)
    # n = 4 rows keeps 2 (Z - T) / n a dyadic rational
    g0 = oracle.mlp_backward(Z0[:4], T[:4], tuple(a[:4] for a in c0), W1, W2, W3)
    g1 = oracle.mlp_backward(Z1[:4], T[:4], tuple(a[:4] for a in c1), W1, W2, W3, rnd=oracle.round_bf16)
    for a, b in zip(g0, g1):
        assert np.array_equal(a, b)


def test_rounded_network_differs_from_exact_by_bf16_error():
    U, params, T = make(seed=5, n=40, d=30, h1=32, h2=32, k=6)
    Z0, _ = oracle.mlp_forward(U, *params)
    Z1, _ = oracle.mlp_forward(U, *params, rnd=oracle.round_bf16)
    rel = np.linalg.norm(Z1 - Z0) / np.linalg.norm(Z0)
    assert 1e-5 < rel < 3e-2


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p = np.array([1.0, 1.0, 1.0, 1.0])
    p1, m, v = oracle.adam_step(p, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    # bias correction makes m^ = g and v^ = g^2 at t = 1
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_gives_constant_steps():
    g = np.array([0.3, -0.7])
    p, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    steps = []
    for t in range(1, 8):
        p_new, m, v = oracle.adam_step(p, g, m, v, t, lr=0.1)
        steps.append(p_new - p)
        p = p_new
    expect = -0.1 * g / (np.abs(g) + 1e-8)
    for s in steps:
        assert np.allclose(s, expect, rtol=1e-12, atol=0)


def _random_rotation(k, rng):
    q, r = np.linalg.qr(rng.standard_normal((k, k)))
    return q * np.sign(np.diag(r))


@pytest.mark.parametrize("seed", [0, 1])
def test_warm_target_planted_rotation_and_centres(seed):
    rng = np.random.default_rng(seed)
    n, k, d = 300, 5, 40
    centres = rng.standard_normal((k, d))
    truth = rng.permutation(n) % k              # planted clusters, cluster c sits at centre g(c)
    g = rng.permutation(k)
    Xh = centres[g[truth]] + 0.3 * rng.standard_normal((n, d))
    Xh /= np.linalg.norm(Xh, axis=1, keepdims=True)
    # an eigenblock whose rotated rows are scaled indicators: Q[:,1:] = diag(s) onehot R^T
    R = _random_rotation(k, rng)
    s = rng.uniform(0.5, 2.0, n)
    Q = np.zeros((n, k + 1))
    Q[:, 0] = 1.0 / np.sqrt(n)
    Q[:, 1:] = (s[:, None] * np.eye(k)[truth]) @ R.T
    T, colmap = oracle.warm_target(Q, R, truth, Xh, centres)
    assert sorted(colmap) == list(range(k))
    assert np.array_equal(colmap, g)
    assert np.allclose(T, np.eye(k)[g[truth]], atol=1e-12)


def test_warm_target_zero_rows_and_empty_cluster():
    rng = np.random.default_rng(2)
    n, k, d = 50, 3, 6
    centres = np.eye(k, d)
    labels = np.arange(n) % 2                   # cluster 2 empty
    Xh = centres[labels] + 0.01 * rng.standard_normal((n, d))
    Q = rng.standard_normal((n, k + 1))
    Q[7, 1:] = 0.0
    T, colmap = oracle.warm_target(Q, np.eye(k), labels, Xh, centres)
    assert np.all(T[7] == 0.0)
    assert colmap[0] == 0 and colmap[1] == 1 and colmap[2] == 2
    nr = np.linalg.norm(T, axis=1)
    assert np.allclose(nr[np.arange(n) != 7], 1.0)


def test_features_average_of_self_and_neighbours():
    import scipy.sparse as sp
    Xh = np.array([[1.0, 0], [0, 1.0], [0.6, 0.8]])
    P = sp.csr_matrix(np.array([[0, 0.5, 0.5], [1.0, 0, 0], [0, 0, 1.0]]))
    U = oracle.mlp_features(Xh, P)
    assert np.allclose(U[0], 0.5 * (Xh[0] + 0.5 * Xh[1] + 0.5 * Xh[2]))
    assert np.allclose(U[2], Xh[2])
