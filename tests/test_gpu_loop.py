"""GPU: scheduling of the clustering loop (Alg. 4, main loop) against the oracle.

The loop queues blocks of tau iterations and runs each check's Discretize and MHC beside the
next block; these cases pin the checks it makes and where it stops: a T_a that is not a
multiple of tau (trailing iterations after the last check), a T_a below tau (no check at all),
and a run without the stopping rules (exactly T_a iterations).
"""
import numpy as np
import pytest

import oracle
from paper_2408_05459_amd import synth
from tests.helpers import ari, oracle_operator

pytestmark = pytest.mark.gpu

_W = {}


def workload():
    if "w" not in _W:
        net, prm = synth.make_config(2, scale=0.03)
        op, ki, ks = oracle_operator(net, prm.K, prm.beta)
        _W["w"] = (net, prm, op)
    return _W["w"]


def run(lib, tau, T_a, early_stop=1):
    net, prm, op = workload()
    s, keep = lib.network(net)
    params = lib.default_params(k=net.k, K=prm.K, alpha=prm.alpha, beta=prm.beta, gamma=prm.gamma, tau=tau,
                                T_i=prm.T_i, T_a=T_a, eps_q=prm.eps_q, knn_mode=prm.knn_mode, q_dtype=prm.q_dtype,
                                early_stop=early_stop)
    lab, info = lib.cluster(s, params)
    return lab.cpu().numpy(), info


@pytest.mark.parametrize("tau,T_a", [(3, 7), (5, 2), (4, 12)])
def test_checks_and_stop_match_oracle(lib, tau, T_a):
    net, prm, op = workload()
    lg, info = run(lib, tau, T_a)
    lr, rep = oracle.cluster(op, net.k, alpha=prm.alpha, gamma=prm.gamma, tau=tau, T_i=prm.T_i, T_a=T_a,
                             eps_q=prm.eps_q)
    print(f"tau={tau} T_a={T_a}: gpu iters {info['iterations']} ({info['stop_reason']}) trace "
          f"{[t for t, _ in info['trace']]}; oracle {rep.iterations} ({rep.reason}) {[t for t, _ in rep.phi_trace]}")
    assert info["iterations"] == rep.iterations
    assert [t for t, _ in info["trace"]] == [t for t, _ in rep.phi_trace]
    for (tg, pg), (tr, pr) in zip(info["trace"], rep.phi_trace):
        assert abs(pg - pr) <= 1e-4 * pr, (tg, pg, pr)
    assert ari(lg, lr) >= 0.99
    if T_a < tau:
        assert info["trace"] == info["trace"][:1] and info["best_t"] == 0


def test_without_stopping_rules_runs_T_a(lib):
    lg, info = run(lib, 5, 15, early_stop=0)
    assert info["iterations"] == 15 and info["stop_reason"] == "max_iter"
    assert [t for t, _ in info["trace"]] == [0, 5, 10, 15]
    best = min(p for _, p in info["trace"])
    assert info["best_phi"] == best
    # the same schedule twice gives the same labels
    lg2, info2 = run(lib, 5, 15, early_stop=0)
    assert np.array_equal(lg, lg2) and info["trace"] == info2["trace"]


def test_warm_block_path_matches_cold_labels_format(lib):
    # a warm block equal to the greedy start's indicators: the loop takes the warm path (no
    # overlapped initial conductance) and must still report the greedy start's conductance
    import torch
    net, prm, op = workload()
    s, keep = lib.network(net)
    y0 = oracle.init_bcm(op, net.k, prm.alpha, prm.T_i)[0]
    Z = np.zeros((net.n, net.k), dtype=np.float32)
    Z[np.arange(net.n), y0] = 1.0
    params = lib.default_params(k=net.k, K=prm.K, alpha=prm.alpha, beta=prm.beta, gamma=prm.gamma, tau=prm.tau,
                                T_i=prm.T_i, T_a=10, eps_q=prm.eps_q, knn_mode=prm.knn_mode, q_dtype=prm.q_dtype)
    lab, info = lib.cluster(s, params, zwarm=torch.from_numpy(Z).cuda())
    phi_cold = oracle.mhc(op, y0, net.k, prm.alpha, prm.gamma)
    assert abs(info["phi_init_cold"] - phi_cold) <= 1e-4 * phi_cold
    assert info["trace"][0][0] == 0
    lg = lab.cpu().numpy()
    assert lg.min() >= 0 and lg.max() < net.k


def test_parameter_study_plumbing(lib):
    """The sweep and convergence drivers on a small hypergraph: one row per value, the trace has
    T + 1 rows, the greedy start's conductance at t = 0 is the run's phi_0."""
    from paper_2408_05459_amd import sweep
    rows = sweep.sweep(lib, 1, 0.2, "beta", [0.0, 0.5])
    assert [r["beta"] for r in rows] == [0.0, 0.5] and all(0 <= r["acc"] <= 1 for r in rows)
    tr = sweep.convergence_trace(lib, 1, 0.2, 6, start="greedy")
    assert [r["t"] for r in tr] == list(range(7))
    net, prm = sweep.synth.make_config(1, scale=0.2)
    s, keep = lib.network(net)
    _, info = lib.cluster(s, lib.default_params(k=net.k, K=prm.K, knn_mode=prm.knn_mode, q_dtype=prm.q_dtype))
    assert abs(tr[0]["phi"] - info["trace"][0][1]) <= 1e-12 * max(1.0, info["trace"][0][1])
    rnd = sweep.convergence_trace(lib, 1, 0.2, 3, start="random")
    assert len(rnd) == 4
