"""GPU parity of the learned warm start (through the C ABI) against the FP64 oracle.

The oracle mirrors the network's rounding points (BF16 operands of every product, FP32
accumulation on the GPU, FP64 in the oracle), so the remaining differences are accumulation
order and the rare activation whose BF16 rounding falls the other way.  Tolerances:
  forward      relative Frobenius error of Zhat <= 1e-4, elementwise <= 2e-3 max|Zhat|; against
               the exact network (no rounding): within a first-order BF16/FP32 error bound;
  gradients    relative Frobenius error <= 1e-3 per parameter tensor;
  Adam         exact gradients (BF16-representable data), updates within 1e-6 relative;
  features     |U_gpu - U_oracle| <= 1e-6 (FP32 sums of unit-norm rows);
  target       |T_gpu - T_oracle| <= 1e-5.
"""
import numpy as np
import pytest

import oracle
from paper_2408_05459_amd import synth, warmstart
from tests.helpers import oracle_operator

pytestmark = pytest.mark.gpu


def torch_mod():
    import torch
    return torch


def rand_params(rng, d, h1, h2, k, scale=1.0):
    W1 = rng.uniform(-1, 1, (d, h1)) / np.sqrt(d) * scale
    W2 = rng.uniform(-1, 1, (h1, h2)) / np.sqrt(h1) * scale
    W3 = rng.uniform(-1, 1, (h2, k)) / np.sqrt(h2) * scale
    b1 = rng.uniform(-0.1, 0.1, h1)
    b2 = rng.uniform(-0.1, 0.1, h2)
    b3 = rng.uniform(-0.1, 0.1, k)
    return [a.astype(np.float32) for a in (W1, b1, W2, b2, W3, b3)]


def upload_u(U, ldu=None):
    torch = torch_mod()
    n, d = U.shape
    ldu = ldu or (d + 3) // 4 * 4
    Ud = torch.zeros((n, ldu), dtype=torch.float32, device="cuda")
    Ud[:, :d] = torch.from_numpy(U.astype(np.float32))
    return Ud


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


SHAPES = [
    # n, d, h1, h2, k: ragged n (not a multiple of the 256-row tile), ragged d and k
    (1000, 100, 64, 48, 30),
    (3001, 512, 256, 256, 30),
    (77, 37, 16, 32, 5),
]


@pytest.mark.parametrize("n,d,h1,h2,k", SHAPES)
def test_forward_parity(lib, n, d, h1, h2, k):
    from paper_2408_05459_amd import binding
    rng = np.random.default_rng(n + d)
    U = rng.uniform(-1, 1, (n, d))
    P = rand_params(rng, d, h1, h2, k)
    ws = binding.WarmStart(lib, d, h1, h2, k, seed=1)
    ws.set(P)
    Z = ws.forward(upload_u(U)).cpu().numpy()
    Zo, _ = oracle.mlp_forward(U.astype(np.float32), *[p.astype(np.float64) for p in P], rnd=oracle.round_bf16)
    assert rel(Z, Zo) <= 1e-4
    assert np.abs(Z - Zo).max() <= 2e-3 * np.abs(Zo).max()
    # the forward values reported by get(0) are the BF16-rounded master weights
    got = ws.get(0)
    for i in (0, 2, 4):
        assert np.array_equal(got[i].astype(np.float64), oracle.round_bf16(P[i]))
    for i in (1, 3, 5):
        assert np.array_equal(got[i], P[i])


def bf16_forward_bound(U, P):
    """Elementwise bound on |Zhat_gpu - Zhat_exact|, Zhat_exact the network in exact arithmetic
    (no rounding anywhere), for the GPU's arithmetic: every product operand rounded to BF16
    (relative error <= u_b = 2^-9), products accumulated in FP32 (gamma_m with u = 2^-24 for m
    terms), the bias added in FP32 (u), relu 1-Lipschitz.  First order in the errors, from the
    exact network's magnitudes:
      D1 = (2 u_b + u_b^2 + gamma_d (1 + u_b)^2) |U| |W1| + u |pre1|,
      E1 = D1 + u_b (|H1| + D1)                                 (H1 rounded to BF16),
      D2 = (1 + u_b)(E1 + gamma_h1 (|H1| + E1)) |W2| + u_b |H1| |W2| + u |pre2|,
      E2 = D2 + u_b (|H2| + D2),
      D3 = (1 + u_b)(E2 + gamma_h2 (|H2| + E2)) |W3| + u_b |H2| |W3| + u |Zhat|."""
    ub, u = 2.0 ** -9, 2.0 ** -24

    def gam(m):
        return m * u / (1.0 - m * u)

    W1, b1, W2, b2, W3, b3 = [np.asarray(p, np.float64) for p in P]
    U = np.asarray(U, np.float64)
    pre1 = U @ W1 + b1
    H1 = np.maximum(pre1, 0.0)
    pre2 = H1 @ W2 + b2
    H2 = np.maximum(pre2, 0.0)
    Z = H2 @ W3 + b3
    D1 = (2 * ub + ub * ub + gam(U.shape[1]) * (1 + ub) ** 2) * (np.abs(U) @ np.abs(W1)) + u * np.abs(pre1)
    E1 = D1 + ub * (H1 + D1)
    D2 = (1 + ub) * ((E1 + gam(W2.shape[0]) * (H1 + E1)) @ np.abs(W2)) + ub * (H1 @ np.abs(W2)) + u * np.abs(pre2)
    E2 = D2 + ub * (H2 + D2)
    D3 = (1 + ub) * ((E2 + gam(W3.shape[0]) * (H2 + E2)) @ np.abs(W3)) + ub * (H2 @ np.abs(W3)) + u * np.abs(Z)
    return Z, D3


@pytest.mark.parametrize("n,d,h1,h2,k", SHAPES)
def test_forward_against_exact_network(lib, n, d, h1, h2, k):
    """The GPU network against the exact one (no rounding, oracle with rnd=None): every output
    within the first-order BF16/FP32 error bound of bf16_forward_bound (times 1.05 for the
    second-order terms), and the oracle's exact network equal to the directly computed one."""
    from paper_2408_05459_amd import binding
    rng = np.random.default_rng(n + d + 1)
    U = rng.uniform(-1, 1, (n, d)).astype(np.float32)
    P = rand_params(rng, d, h1, h2, k)
    ws = binding.WarmStart(lib, d, h1, h2, k, seed=1)
    ws.set(P)
    Z = ws.forward(upload_u(U)).cpu().numpy().astype(np.float64)
    Zx, _ = oracle.mlp_forward(U.astype(np.float64), *[p.astype(np.float64) for p in P], rnd=None)
    Zb, B = bf16_forward_bound(U, P)
    assert np.allclose(Zx, Zb, rtol=1e-12, atol=1e-12)
    err = np.abs(Z - Zx)
    print(f"n={n} d={d}: max |Z - Z_exact| {err.max():.3e}, max bound {B.max():.3e}, "
          f"max err/bound {(err / B).max():.3f}")
    assert (err <= 1.05 * B).all()


@pytest.mark.parametrize("n,d,h1,h2,k", SHAPES)
def test_backward_parity(lib, n, d, h1, h2, k):
    from paper_2408_05459_amd import binding
    torch = torch_mod()
    rng = np.random.default_rng(7 * n + d)
    U = rng.uniform(-1, 1, (n, d))
    P = rand_params(rng, d, h1, h2, k, scale=2.0)
    T = rng.standard_normal((n, k))
    ws = binding.WarmStart(lib, d, h1, h2, k, seed=2)
    ws.set(P)
    Zd = ws.forward(upload_u(U), keep_acts=True)
    Td = torch.from_numpy(T.astype(np.float32)).cuda()
    loss = ws.backward(Zd, Td)
    G = ws.get(1)
    P64 = [p.astype(np.float64) for p in P]
    Zo, cache = oracle.mlp_forward(U.astype(np.float32), *P64, rnd=oracle.round_bf16)
    To = T.astype(np.float32).astype(np.float64)
    Go = oracle.mlp_backward(Zo, To, cache, P64[0], P64[2], P64[4], rnd=oracle.round_bf16)
    assert abs(loss - oracle.mlp_loss(Zo, To)) <= 1e-5 * oracle.mlp_loss(Zo, To)
    names = ["W1", "b1", "W2", "b2", "W3", "b3"]
    for nm, g, go in zip(names, G, Go):
        assert g.shape == go.shape, nm
        assert rel(g, go) <= 1e-3, (nm, rel(g, go))


def exact_case(seed):
    """Sparse small-integer data on which every BF16 rounding point is exact (checked)."""
    rng = np.random.default_rng(seed)
    n, d, h1, h2, k = 4, 16, 16, 16, 4

    def sparse(shape):
        return (rng.integers(-1, 2, shape) * (rng.random(shape) < 0.3)).astype(np.float64)

    U = sparse((n, d))
    W1, W2, W3 = sparse((d, h1)), sparse((h1, h2)), sparse((h2, k))
    b1 = rng.integers(0, 2, h1).astype(np.float64)
    b2 = rng.integers(0, 2, h2).astype(np.float64)
    b3 = np.zeros(k)
    T = rng.integers(-2, 3, (n, k)).astype(np.float64)
    P = [W1, b1, W2, b2, W3, b3]
    Z0, c0 = oracle.mlp_forward(U, *P)
    Z1, c1 = oracle.mlp_forward(U, *P, rnd=oracle.round_bf16)
    g0 = oracle.mlp_backward(Z0, T, c0, W1, W2, W3)
    g1 = oracle.mlp_backward(Z1, T, c1, W1, W2, W3, rnd=oracle.round_bf16)
    exact = np.array_equal(Z0, Z1) and all(np.array_equal(a, b) for a, b in zip(g0, g1))
    nonzero = all(np.any(g != 0) for g in g0[::2])
    return exact and nonzero, (U, P, T, g0)


def test_adam_steps_parity(lib):
    from paper_2408_05459_amd import binding
    torch = torch_mod()
    seed = next(s for s in range(100) if exact_case(s)[0])
    _, (U, P, T, G) = exact_case(seed)
    ws = binding.WarmStart(lib, 16, 16, 16, 4, seed=3)
    ws.set([p.astype(np.float32) for p in P])
    Zd = ws.forward(upload_u(U), keep_acts=True)
    ws.backward(Zd, torch.from_numpy(T.astype(np.float32)).cuda())
    for g, go in zip(ws.get(1), G):
        assert np.array_equal(g.astype(np.float64), go)
    lr = 0.05
    p_o = [p.copy() for p in P]
    m_o = [np.zeros_like(p) for p in P]
    v_o = [np.zeros_like(p) for p in P]
    for t in (1, 2):                       # two steps with the stored gradients: bias corrections at t = 1, 2
        ws.step(lr)
        for i in range(6):
            p_o[i], m_o[i], v_o[i] = oracle.adam_step(p_o[i], G[i], m_o[i], v_o[i], t, lr)
        got = ws.get(2)
        for a, b in zip(got, p_o):
            assert np.allclose(a, b, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("cfg", [5, 4, 3])
def test_features_parity(lib, cfg):
    torch = torch_mod()
    if cfg == 5:
        net, prm = synth.make_warm_graph(3000, 5003, k=30, d=512)
    else:
        net, prm = synth.make_config(cfg, scale={4: 0.002, 3: 0.006}[cfg])
    s, keep = lib.network(net)
    # the features use the topology walk only; the KNN part comes from the oracle lists
    op_o, ki, ks = oracle_operator(net, prm.K, prm.beta)
    idx = torch.from_numpy(ki.astype(np.int32)).cuda()
    sim = torch.from_numpy(ks.astype(np.float32)).cuda()
    op = lib.build_operator(s, idx, sim, prm.K, prm.beta, "f32")
    U = lib.ws_features(op, keep[-1]).cpu().numpy()
    Xh, _ = oracle.normalize_rows(net.X)
    P_N = oracle.topology_transition(net.kind, net.n, net.ptrs, net.idxs, net.m)["P_N"]
    Uo = oracle.mlp_features(Xh, P_N)
    d = net.X.shape[1]
    assert np.abs(U[:, :d] - Uo).max() <= 1e-6
    assert np.all(U[:, d:(d + 3) // 4 * 4] == 0)


def test_features_zero_rows_and_isolated_nodes(lib):
    # the n = 2000 binary hypergraph has nodes in no hyperedge (delta = 0); two rows are zeroed
    torch = torch_mod()
    net, prm = synth.make_config(1, scale=1.0)
    net.X[[3, 50]] = 0.0
    s, keep = lib.network(net)
    op_o, ki, ks = oracle_operator(net, prm.K, prm.beta)
    op = lib.build_operator(s, torch.from_numpy(ki.astype(np.int32)).cuda(),
                            torch.from_numpy(ks.astype(np.float32)).cuda(), prm.K, prm.beta, "f32")
    U = lib.ws_features(op, keep[-1]).cpu().numpy()
    d = net.X.shape[1]
    Xh, _ = oracle.normalize_rows(net.X)
    topo = oracle.topology_transition(net.kind, net.n, net.ptrs, net.idxs, net.m)
    P_N, delta = topo["P_N"], topo["delta"]
    Uo = oracle.mlp_features(Xh, P_N)
    assert np.abs(U[:, :d] - Uo).max() <= 1e-6
    iso = np.flatnonzero(delta == 0)
    assert iso.size > 0
    assert np.allclose(U[iso, :d], 0.5 * Xh[iso], atol=1e-7)


@pytest.mark.parametrize("qdt", ["f32", "f64"])
def test_target_parity(lib, qdt):
    torch = torch_mod()
    rng = np.random.default_rng(11)
    n, k, d = 2500, 30, 64
    Q = rng.standard_normal((n, k + 1))
    Q[[5, 99], 1:] = 0.0                   # zero rows of the k-column block stay zero
    R, _ = np.linalg.qr(rng.standard_normal((k, k)))
    centres = rng.standard_normal((k, d))
    labels = rng.permutation(n) % k
    Xh = centres[labels] + 0.5 * rng.standard_normal((n, d))
    colmap = oracle.centre_map(labels, Xh, centres)
    Y = oracle.rotated_block(Q[:, 1:], R)
    To = np.zeros_like(Y)
    To[:, colmap] = Y
    dt = torch.float64 if qdt == "f64" else torch.float32
    Qd = torch.zeros((n, 32), dtype=dt, device="cuda")
    Qd[:, :k + 1] = torch.from_numpy(Q)
    T = lib.ws_target(Qd[:, 1:], k, R, colmap).cpu().numpy()
    assert np.abs(T - To).max() <= 1e-5
    assert np.all(T[[5, 99]] == 0)


def test_target_rejects_non_permutation(lib):
    torch = torch_mod()
    from paper_2408_05459_amd import binding
    Q = torch.zeros((10, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(binding.AnckaError):
        lib.ws_target(Q[:, 1:], 3, np.eye(3), [0, 0, 2])


def test_training_is_deterministic_and_reduces_loss(lib):
    torch = torch_mod()
    exs = warmstart.make_examples(lib, 3000, [5101, 5102, 5103, 5104])
    ws_a, log_a = warmstart.train(lib, exs, 512, 30, epochs=15, lr=2e-3, seed=9)
    ws_b, log_b = warmstart.train(lib, exs, 512, 30, epochs=15, lr=2e-3, seed=9)
    assert log_a.epoch_loss == log_b.epoch_loss
    for a, b in zip(ws_a.get(2), ws_b.get(2)):
        assert np.array_equal(a, b)
    assert log_a.epoch_loss[-1] < 0.5 * log_a.epoch_loss[0]
    torch.cuda.synchronize()


def test_ws_argument_errors(lib):
    from paper_2408_05459_amd import binding
    with pytest.raises(binding.AnckaError):
        binding.WarmStart(lib, 512, 250, 256, 30)      # h1 not a multiple of 16
    with pytest.raises(binding.AnckaError):
        binding.WarmStart(lib, 512, 256, 256, 65)      # k > 64
    ws = binding.WarmStart(lib, 8, 16, 16, 3)
    torch = torch_mod()
    U = torch.zeros((5, 8), dtype=torch.float32, device="cuda")
    Z = ws.forward(U)                                  # no activations kept
    with pytest.raises(binding.AnckaError):
        ws.backward(Z, torch.zeros_like(Z))
