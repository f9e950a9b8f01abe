"""GPU edge cases and full-size sampled parity (through the C ABI, against the FP64 oracle).

Edge cases: zero attribute rows in every KNN mode, K = n - 1, the smallest networks, an empty
cluster in the starting block, argument errors.  Full size: the n = 2.5M benchmark graph in the
launch configuration the benchmark times, with the KNN lists of sampled rows checked against the
oracle's exact FP64 search over all n candidates, and P 1 = 1 over every row.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2408_05459_amd import synth
from tests.helpers import check_knn_rows, gamma_d, oracle_operator

pytestmark = pytest.mark.gpu


def torch_mod():
    import torch
    return torch


def tol_for(mode, d):
    return 2 * gamma_d(d, 2.0 ** -53 if mode == "f64" else 2.0 ** -24)


def upload(X, mode):
    from paper_2408_05459_amd.binding import upload_attributes
    return upload_attributes(X, {"f64": "f64", "f32": "f32", "bf16": "bf16"}[mode])


def gmm(n, d, k, seed, dtype):
    rng = np.random.default_rng(seed)
    labels = synth.planted_labels(n, k, rng)
    cen = synth.gmm_centres(k, d, 2.0, rng)
    return synth.gmm_attributes(labels, cen, rng, dtype), labels


@pytest.mark.parametrize("mode", ["f64", "f32", "bf16"])
def test_knn_zero_rows(lib, mode):
    X, _ = gmm(700, 64, 5, 1, "bf16" if mode == "bf16" else "f32")
    X = np.asarray(X, dtype=np.float64 if mode == "f64" else np.float32)
    zero = [0, 13, 699]
    X[zero] = 0
    K = 8
    idx, sim, st = lib.knn(upload(X, mode), K, mode)
    gi, gs = idx.cpu().numpy(), sim.cpu().numpy()
    assert st.zero_rows == len(zero)
    for z in zero:
        assert np.all(gi[z] == -1) and np.all(gs[z] == 0)
    assert not np.isin(gi, zero).any()
    rows = np.setdiff1d(np.arange(X.shape[0]), zero)
    check_knn_rows(X, rows, gi[rows], gs[rows], K, tol_for(mode, X.shape[1]))


@pytest.mark.parametrize("mode,n,K", [("f64", 40, 39), ("f32", 17, 16), ("bf16", 17, 16), ("bf16", 130, 16)])
def test_knn_all_other_rows(lib, mode, n, K):
    X, _ = gmm(n, 24, 3, 2, "bf16" if mode == "bf16" else "f32")
    X = np.asarray(X, dtype=np.float64 if mode == "f64" else np.float32)
    idx, sim, st = lib.knn(upload(X, mode), K, mode)
    gi, gs = idx.cpu().numpy(), sim.cpu().numpy()
    check_knn_rows(X, np.arange(n), gi, gs, K, tol_for(mode, X.shape[1]))
    if K == n - 1:
        for i in range(n):
            assert sorted(gi[i].tolist()) == [j for j in range(n) if j != i]


def test_knn_argument_errors(lib):
    from paper_2408_05459_amd import binding
    X = upload(np.ones((5, 8), dtype=np.float32), "f32")
    for K in (0, 5):                         # K must lie in [1, n-1]
        with pytest.raises(binding.AnckaError):
            lib.knn(X, K, "f32")
    with pytest.raises(binding.AnckaError):
        lib.knn(upload(np.ones((1, 8), dtype=np.float32), "f32"), 1, "f32")   # n < 2
    with pytest.raises(binding.AnckaError):
        lib.knn(upload(np.ones((80, 8), dtype=np.float32), "f32"), 65, "f32")  # K > 64


def test_mhc_rejects_labels_out_of_range(lib):
    torch = torch_mod()
    from paper_2408_05459_amd import binding
    net, prm = synth.make_config(1, scale=0.1)
    op_o, ki, ks = oracle_operator(net, prm.K, prm.beta)
    s, keep = lib.network(net)
    op = lib.build_operator(s, torch.from_numpy(ki.astype(np.int32)).cuda(),
                            torch.from_numpy(ks).cuda(), prm.K, prm.beta, prm.q_dtype)
    bad = torch.from_numpy(np.where(np.arange(net.n) == 5, net.k, net.labels).astype(np.int32)).cuda()
    with pytest.raises(binding.AnckaError):
        op.mhc(bad, net.k, prm.alpha, prm.gamma)


def test_initial_block_with_empty_cluster(lib):
    torch = torch_mod()
    net, prm = synth.make_config(1, scale=0.3)
    op_o, ki, ks = oracle_operator(net, prm.K, prm.beta)
    s, keep = lib.network(net)
    op = lib.build_operator(s, torch.from_numpy(ki.astype(np.int32)).cuda(),
                            torch.from_numpy(ks).cuda(), prm.K, prm.beta, prm.q_dtype)
    y = net.labels.copy()
    y[y == 2] = 3                            # cluster 2 empty
    C = np.concatenate([np.full((net.n, 1), 1 / math.sqrt(net.n)), oracle.normalized_bcm(y, net.k)], axis=1)
    Qr = oracle.initial_q(C)
    Q = op.initial_block(net.k, labels=torch.from_numpy(y.astype(np.int32)).cuda())
    kp = net.k + 1
    Qg = Q.cpu().numpy()[:, :kp]
    assert np.abs(Qg - Qr).max() <= 1e-11
    assert np.abs(Qg.T @ Qg - np.eye(kp)).max() <= 1e-12


def test_cluster_two_clusters_and_tiny_network(lib):
    # k = 2 on a small planted hypergraph: the smallest non-trivial block (3 columns)
    torch = torch_mod()
    from paper_2408_05459_amd import binding
    rng = np.random.default_rng(3)
    n, k = 120, 2
    labels = synth.planted_labels(n, k, rng)
    sizes = rng.integers(2, 6, 200)
    ptr, idx = synth.hypergraph_incidence(labels, k, sizes, 0.9, rng)
    X = synth.gmm_attributes(labels, synth.gmm_centres(k, 16, 3.0, rng), rng, "f32").astype(np.float64)
    net = synth.Network(synth.HYPERGRAPH, n, k, X, "f64", [ptr], [idx], m=len(sizes), labels=labels, name="tiny")
    s, keep = lib.network(net)
    params = lib.default_params(k=k, K=5, knn_mode="f64", q_dtype="f64")
    lab, info = lib.cluster(s, params)
    lg = lab.cpu().numpy()
    op_o, ki, ks = oracle_operator(net, 5, 0.5)
    lr, rep = oracle.cluster(op_o, k)
    from tests.helpers import ari
    assert ari(lg, lr) >= 0.99
    phi_g = oracle.mhc(op_o, lg, k, 0.2, 3)
    assert abs(phi_g - rep.best_phi) <= 1e-4 * abs(rep.best_phi)
    bad = lib.default_params(k=n + 1, K=5, knn_mode="f64", q_dtype="f64")
    with pytest.raises(binding.AnckaError):
        lib.cluster(s, bad)


@pytest.mark.timeout(600)
def test_full_size_benchmark_graph_sampled(lib):
    """n = 2.5M graph of the benchmark: BF16 KNN of 40 sampled rows against the oracle's exact
    search over all rows; P 1 = 1 for the operator built from the GPU lists."""
    torch = torch_mod()
    net, prm = synth.make_config(4, scale=1.0)
    X = upload(net.X, "bf16")
    idx, sim, st = lib.knn(X, prm.K, prm.knn_mode)
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    rows = np.sort(rng.choice(net.n, size=40, replace=False))
    gi = idx[torch.from_numpy(rows).cuda()].cpu().numpy()
    gs = sim[torch.from_numpy(rows).cuda()].cpu().numpy()
    swaps = check_knn_rows(net.X, rows, gi, gs, prm.K, tol_for("bf16", net.d))
    assert swaps <= 1
    s, keep = lib.network(net)
    op = lib.build_operator(s, idx, sim, prm.K, prm.beta, prm.q_dtype)
    del X
    ones = torch.ones((net.n, 52), dtype=torch.float32, device="cuda")
    P1 = op.apply(ones)
    assert float((P1 - 1.0).abs().max()) <= 1e-5


def test_discretize_cluster_beyond_2_pow_23_rows(lib):
    """One cluster of 2^23 + 4096 rows equal to (1, 0): the fixed-point cluster sum would be
    2^63 + 2^52 at the scale 2^40; the scale chosen from n keeps it exact, so the cluster mean
    is (1, 0) and the objective is the oracle's."""
    import torch
    import oracle
    n, k = (1 << 23) + 4096, 2
    T = torch.zeros((n, k), dtype=torch.float32, device="cuda")
    T[:, 0] = 1.0
    lg, Rg, objg, itg = lib.discretize(T, k)
    lr, Rr, objr, itr = oracle.discretize(np.tile([1.0, 0.0], (n, 1)))
    assert not lg.any().item() and not lr.any()
    assert np.abs(Rg - Rr).max() <= 1e-12 and itg == itr
    assert abs(objg - objr) <= 1e-6 and abs(objr - (n - 2.0)) <= 1e-6


def _messy_csr(n, ptr, idx, rng):
    """The same undirected graph given as a messy directed CSR: of each edge pair (i, j),
    (j, i) a random one of the two directions is dropped half of the time, 3% of the entries
    are repeated, self loops are added at 2% of the nodes, and every row's columns are
    shuffled.  The method reads it as the original simple graph (Sec. 6.1: reverse edges
    added; A is binary; self loops dropped)."""
    rows = np.repeat(np.arange(n), np.diff(ptr))
    cols = np.asarray(idx, dtype=np.int64)
    lo, hi = np.minimum(rows, cols), np.maximum(rows, cols)
    drop = rng.random(rows.shape[0]) < 0.5
    keep_dir = ((lo * 7919 + hi) % 2 == 0)            # the direction kept, one per pair
    keep = ~drop | ((rows < cols) == keep_dir)
    r, c = rows[keep], cols[keep]
    dup = rng.random(r.shape[0]) < 0.03
    loops = rng.choice(n, size=max(1, n // 50), replace=False)
    r = np.concatenate([r, r[dup], loops])
    c = np.concatenate([c, c[dup], loops])
    order = np.lexsort((rng.random(r.shape[0]), r))
    r, c = r[order], c[order]
    p = np.zeros(n + 1, dtype=np.int64)
    np.add.at(p, r + 1, 1)
    return np.cumsum(p), c.astype(np.int32)


@pytest.mark.parametrize("cfg,scale", [(1, 0.5), (3, 0.006), (4, 0.002)])
def test_operator_parity_messy_topology(lib, cfg, scale):
    """Directed edges, duplicate entries, self loops and unsorted rows (graph and multiplex),
    repeated hyperedge members (hypergraph): the GPU operator equals the oracle's, which reads
    them as Sec. 6.1 and Sec. 2 define the simple network."""
    import dataclasses
    torch = torch_mod()
    net, prm = synth.make_config(cfg, scale=scale)
    rng = np.random.default_rng(100 + cfg)
    if net.kind == synth.HYPERGRAPH:
        ptr, idx = net.ptrs[0], net.idxs[0]
        sizes = np.diff(ptr)
        members = np.split(idx, ptr[1:-1])
        new = []
        for e in members:
            extra = e[rng.random(e.shape[0]) < 0.2]
            new.append(rng.permutation(np.concatenate([e, extra, e[:1]])))
        p2 = np.zeros(len(new) + 1, dtype=np.int64)
        p2[1:] = np.cumsum([len(e) for e in new])
        messy = dataclasses.replace(net, ptrs=[p2], idxs=[np.concatenate(new).astype(np.int32)])
        assert (np.diff(p2) > sizes).all()
    else:
        ps, ix = [], []
        for p, i in zip(net.ptrs, net.idxs):
            p2, i2 = _messy_csr(net.n, p, i, rng)
            ps.append(p2)
            ix.append(i2)
        messy = dataclasses.replace(net, ptrs=ps, idxs=ix)
    op_clean, ki, ks = oracle_operator(net, prm.K, prm.beta)
    op_messy, _, _ = oracle_operator(messy, prm.K, prm.beta, knn=(ki, ks))
    # the oracle reads both as the same network
    assert np.array_equal(op_clean.delta, op_messy.delta) and np.array_equal(op_clean.beta, op_messy.beta)
    s, keep = lib.network(messy)
    gop = lib.build_operator(s, torch.from_numpy(ki.astype(np.int32)).cuda(),
                             torch.from_numpy(ks.astype(np.float64 if prm.q_dtype == "f64" else np.float32)).cuda(),
                             prm.K, prm.beta, prm.q_dtype)
    info = gop.info()
    assert np.array_equal(info["delta"], op_messy.delta.astype(np.int64))
    assert np.array_equal(info["beta"], op_messy.beta)
    kp = net.k + 1
    ld = kp + (-kp) % (2 if prm.q_dtype == "f64" else 4)
    Qh = np.zeros((net.n, ld))
    Qh[:, :kp] = rng.standard_normal((net.n, kp))
    dt = torch.float64 if prm.q_dtype == "f64" else torch.float32
    Q = torch.from_numpy(Qh).to(dt).cuda()
    Zg = gop.apply(Q).cpu().double().numpy()[:, :kp]
    Qd = Q.cpu().double().numpy()[:, :kp]
    Zr = oracle.apply_P(op_messy, Qd)
    Zabs = oracle.apply_P(op_messy, np.abs(Qd))
    assert (np.abs(Zg - Zr) / Zabs).max() <= (1e-12 if prm.q_dtype == "f64" else 1e-5)


@pytest.mark.parametrize("mode", ["f32", "bf16"])
def test_knn_near_ties_take_exact_recompute(lib, mode):
    """24 rows equal to one base vector except that row g has coordinate g raised by 2, 3 or 4
    units of 1/128 (all values BF16): every such row's 23 group neighbours lie within 2.6e-6
    of one another, below the candidate scores' resolution (about 8.6e-6 at d = 32), so no 2K
    candidate list of these rows can prove its top K and each is recomputed exactly in FP64.
    The seeded design keeps the exact order's gaps at 4.9e-14 or more, six times the FP64 tie
    tolerance (products of BF16 values and their sums over 32 terms are exact in FP64, so both
    sides compute the same cosines).  The lists must equal the oracle's, order included."""
    d, K, G = 32, 10, 24
    rng = np.random.default_rng(43)
    base = 1.0 + rng.choice(110, size=d, replace=False) / 128.0
    group = np.tile(base, (G, 1))
    group[np.arange(G), np.arange(G)] += rng.choice([2, 3, 4], size=G) / 128.0
    bg, _ = gmm(700, d, 6, 12, "bf16" if mode == "bf16" else "f32")
    X = np.concatenate([bg[:300], group, bg[300:]]).astype(np.float32)
    if mode == "bf16":
        assert np.array_equal(synth.round_to_bf16(X), X)
    S = oracle.cosine_rows(X, np.arange(300, 300 + G))
    top = -np.sort(-S, axis=1)
    assert (top[:, 0] - top[:, 2 * K - 1]).max() < 3e-6
    assert np.diff(-top[:, :2 * K + 1], axis=1).min() >= 6 * tol_for("f64", d)
    idx, sim, st = lib.knn(upload(X, mode), K, mode)
    gi, gs = idx.cpu().numpy(), sim.cpu().numpy()
    print(f"{mode}: uncertified {st.uncertified_rows} recomputed {st.recomputed_rows}")
    assert st.uncertified_rows >= G and st.recomputed_rows == st.uncertified_rows
    swaps = check_knn_rows(X, np.arange(X.shape[0]), gi, gs, K, tol_for("f64", d))
    assert swaps == 0
    ref_i, _ = oracle.knn(X, K, rows=np.arange(300, 300 + G))
    assert np.array_equal(gi[300:300 + G], ref_i)


@pytest.mark.parametrize("mode", ["f32", "bf16"])
def test_knn_k40_near_ties_take_exact_recompute(lib, mode):
    """K = 40 (candidate lists of 80): 90 rows equal to one base vector except for one raised
    coordinate each (2 to 6 units of 1/128), all within 5e-6 of one another in cosine, below the
    candidate scores' resolution at d = 96, so every one of them is recomputed exactly; the
    recompute's four per-wave lists of 40 are merged into the final list.  BF16 values: the
    products and their sums are exact in FP64, so both sides compute identical cosines and
    break equal ones by index; the lists must equal the oracle's, order included."""
    d, K, G = 96, 40, 90
    rng = np.random.default_rng(40)
    base = 1.0 + rng.choice(110, size=d, replace=False) / 128.0
    group = np.tile(base, (G, 1))
    group[np.arange(G), np.arange(G)] += rng.choice([2, 3, 4, 5, 6], size=G) / 128.0
    bg, _ = gmm(600, d, 6, 13, "bf16")
    X = np.concatenate([bg[:250], group, bg[250:]]).astype(np.float32)
    assert np.array_equal(synth.round_to_bf16(X), X)
    rows = np.arange(250, 250 + G)
    S = oracle.cosine_rows(X, rows)
    top = -np.sort(-S, axis=1)
    assert (top[:, 0] - top[:, 2 * K - 1]).max() < 5e-6
    idx, sim, st = lib.knn(upload(X, mode), K, mode)
    gi, gs = idx.cpu().numpy(), sim.cpu().numpy()
    print(f"{mode}: uncertified {st.uncertified_rows}")
    assert st.uncertified_rows >= G and st.recomputed_rows == st.uncertified_rows
    ref_i, _ = oracle.knn(X, K, rows=rows)
    assert np.array_equal(gi[rows], ref_i)
    check_knn_rows(X, np.arange(X.shape[0]), gi, gs, K, tol_for("f64", d))


@pytest.mark.parametrize("mode,K", [("f32", 50), ("bf16", 50), ("f32", 64), ("bf16", 64)])
def test_knn_long_lists(lib, mode, K):
    """K = 50 (the paper's value for attributed graphs and multiplex graphs, Sec. 8.1) and the
    largest K = 64: candidate lists of 100 and 128 kept in global memory by the BF16 passes,
    rescored and certified; every row against the oracle (FP64 tie tolerance, no set
    differences)."""
    X, _ = gmm(1500, 128 if mode == "bf16" else 40, 8, 14, "bf16" if mode == "bf16" else "f32")
    X = np.asarray(X, dtype=np.float32)
    X[[3, 700]] = 0.0
    idx, sim, st = lib.knn(upload(X, mode), K, mode)
    gi, gs = idx.cpu().numpy(), sim.cpu().numpy()
    print(f"{mode} K={K}: uncertified {st.uncertified_rows}")
    assert st.zero_rows == 2 and (gi[[3, 700]] == -1).all()
    rows = np.setdiff1d(np.arange(X.shape[0]), [3, 700])
    swaps = check_knn_rows(X, rows, gi[rows], gs[rows], K, tol_for("f64", X.shape[1]))
    assert swaps == 0


def test_orth_iter_takes_shifted_cholesky(lib):
    """FP64 block whose third and fourth columns agree to 1e-9: the Gram of Z = P Q has a
    pivot ratio near 1e-18, below the 1e-15 at which the plain Cholesky factorisation is
    refused, so the step takes the shifted factorisation and its second pass (shifted
    CholeskyQR3).  Q must still be the unique QR factor with positive diagonal (the oracle's
    Householder QR), to the accuracy its condition number (about 1e9) allows."""
    torch = torch_mod()
    net, prm = synth.make_config(1, scale=0.5)
    op_o, ki, ks = oracle_operator(net, prm.K, prm.beta)
    s, keep = lib.network(net)
    op = lib.build_operator(s, torch.from_numpy(ki.astype(np.int32)).cuda(), torch.from_numpy(ks).cuda(),
                            prm.K, prm.beta, "f64")
    rng = np.random.default_rng(21)
    kp = net.k + 1
    Q0 = rng.standard_normal((net.n, kp))
    Q0[:, 3] = Q0[:, 2] + 1e-9 * rng.standard_normal(net.n)
    Z = oracle.apply_P(op_o, Q0)
    # the plain factorisation's pivots (the kernel's rule): one falls below 1e-15 of its diagonal
    G = Z.T @ Z
    ratios = []
    A = G.copy()
    for j in range(kp):
        ratios.append(A[j, j] / G[j, j])
        A[j + 1:, j + 1:] -= np.outer(A[j + 1:, j], A[j, j + 1:]) / A[j, j]
    assert min(ratios) < 1e-15
    ld = 8
    Qt = torch.zeros((net.n, ld), dtype=torch.float64, device="cuda")
    Qt[:, :kp] = torch.from_numpy(Q0).cuda()
    R, dq = op.orth_iter(Qt, kp, 1)
    Qg = Qt.cpu().numpy()[:, :kp]
    Qr, Rr = oracle.qr_pos(Z)
    assert np.abs(Qg.T @ Qg - np.eye(kp)).max() <= 1e-12
    assert np.abs(Qg @ R - Z).max() <= 1e-12 * np.abs(Z).max()
    assert np.abs(Qg[:, :3] - Qr[:, :3]).max() <= 1e-11
    assert np.abs(Qg - Qr).max() <= 1e-5
