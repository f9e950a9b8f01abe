"""GPU: approximate KNN with the IVF coarse quantiser (ancka_knn_ivf) against the exact oracle.

The IVF search is approximate by design; it is judged by recall against the exact KNN lists and
by the clustering it leads to against the exact pipeline.  Exact pins: probing every list is the
exact search; every returned similarity is the row pair's exact cosine; lists are ordered.
"""
import numpy as np
import pytest

import oracle
from paper_2408_05459_amd import synth
from tests.helpers import ari, check_knn_rows, gamma_d, oracle_operator

pytestmark = pytest.mark.gpu

_W = {}


def workload(scale=0.002):
    if scale not in _W:
        net, prm = synth.make_config(4, scale=scale)
        _W[scale] = (net, prm, oracle.knn(net.X, prm.K))
    return _W[scale]


def run_ivf(lib, net, K, nlist, nprobe):
    from paper_2408_05459_amd.binding import upload_attributes
    X = upload_attributes(net.X, "bf16")
    idx, sim, st = lib.knn_ivf(X, K, nlist, nprobe)
    return idx.cpu().numpy(), sim.cpu().numpy(), st


def recall(gi, ki):
    hits = sum(len(set(a[a >= 0]) & set(b[b >= 0])) for a, b in zip(gi, ki))
    return hits / max(1, int((ki >= 0).sum()))


def test_ivf_probing_every_list_is_exact(lib):
    net, prm, (ki, ks) = workload()
    gi, gs, st = run_ivf(lib, net, prm.K, 16, 16)
    swaps = check_knn_rows(net.X, np.arange(net.n), gi, gs, prm.K, 2 * gamma_d(net.d, 2.0 ** -53))
    assert swaps == 0
    assert st.sym_pairs >= net.n * net.n


@pytest.mark.parametrize("nlist,nprobe,min_recall", [(32, 8, 0.95), (64, 4, 0.85)])
def test_ivf_recall_and_exact_similarities(lib, nlist, nprobe, min_recall):
    net, prm, (ki, ks) = workload()
    gi, gs, st = run_ivf(lib, net, prm.K, nlist, nprobe)
    r = recall(gi, ki)
    print(f"nlist {nlist} nprobe {nprobe}: recall {r:.4f}, pairs scored {st.sym_pairs / net.n ** 2:.3f} of n^2")
    assert r >= min_recall
    assert st.sym_pairs < net.n * net.n
    # every returned neighbour carries its exact cosine, lists ordered, no self, no duplicates
    rows = np.arange(0, net.n, 7)
    S = oracle.cosine_rows(net.X, rows)
    for t, i in enumerate(rows):
        g = gi[i][gi[i] >= 0]
        assert i not in g and len(set(g)) == len(g)
        assert np.all(np.abs(gs[i][:len(g)] - S[t][g]) <= 1e-7 * np.abs(S[t][g]) + 1e-7)
        assert np.all(np.diff(gs[i][:len(g)]) <= 1e-7)


def test_ivf_clustering_against_the_exact_pipeline(lib):
    """The whole method with IVF lists (knn_mode 'ivf') against the oracle's run on the exact KNN
    graph of the same workload: labels and conductance close to the exact pipeline's."""
    net, prm, (ki, ks) = workload(0.02)
    op, _, _ = oracle_operator(net, prm.K, prm.beta, knn=(ki, ks))
    lr, rep = oracle.cluster(op, net.k, alpha=prm.alpha, gamma=prm.gamma, tau=prm.tau, T_i=prm.T_i, T_a=prm.T_a,
                             eps_q=prm.eps_q)
    s, keep = lib.network(net)
    params = lib.default_params(k=net.k, K=prm.K, knn_mode="ivf", q_dtype=prm.q_dtype)
    params.ivf_nlist = 256
    params.ivf_nprobe = 16
    lg, info = lib.cluster(s, params)
    lg = lg.cpu().numpy()
    phi_g = oracle.mhc(op, lg, net.k, prm.alpha, prm.gamma)
    a = ari(lg, lr)
    print(f"IVF clustering n={net.n}: ARI vs exact pipeline {a:.4f}, phi (exact operator) {phi_g:.6f} vs "
          f"{rep.best_phi:.6f}, KNN {info['phase_ms']['knn']:.1f} ms")
    assert a >= 0.98
    assert abs(phi_g - rep.best_phi) <= 1e-3 * rep.best_phi


def test_ivf_argument_errors(lib):
    from paper_2408_05459_amd import binding
    net, prm, _ = workload()
    from paper_2408_05459_amd.binding import upload_attributes
    X = upload_attributes(net.X, "bf16")
    for nlist, nprobe in ((0, 1), (16, 17), (net.n + 1, 1), (64, 65), (5000, 1)):
        with pytest.raises(binding.AnckaError):
            lib.knn_ivf(X, prm.K, nlist, nprobe)
    with pytest.raises(binding.AnckaError):
        lib.knn_ivf(X.float(), prm.K, 16, 4)


def test_ivf_recall_on_weak_clusters(lib):
    """Weakly separated clusters (the study's hard graph at n = 20k): neighbours spread over more
    lists, so probing 4 of 64 lists misses some; recall grows with the lists probed and reaches
    1 when every list is probed."""
    from paper_2408_05459_amd import sweep
    net, prm = sweep.hard_graph(n=20000)
    ki, _ = oracle.knn(net.X, prm.K)
    rec = []
    for nprobe in (2, 8, 64):
        gi, gs, st = run_ivf(lib, net, prm.K, 64, nprobe)
        rec.append(recall(gi, ki))
    print(f"hard graph n={net.n}, 64 lists: recall at nprobe 2/8/64 = {rec}")
    assert rec[0] <= rec[1] <= rec[2] and rec[2] >= 0.999 and rec[1] >= 0.5
