"""Parameter sweeps and convergence traces of the clustering method on the synthetic workloads.

The paper studies how the result depends on K, beta, gamma (Sec. 8.3) and how the conductance
phi_t and the quality evolve over the iterations with early termination switched off and a check
at every iteration, for the greedy start and for a random start (Sec. 8.4).  Its datasets are not
available; these functions run the same studies on the seeded planted-partition workloads, whose
planted labels stand in for the ground truth.  Every step runs on the GPU through the C ABI.

Quality against the planted labels: Acc (best one-to-one matching of clusters to classes,
Hungarian method), macro F1 under that matching, NMI and ARI.
"""
from __future__ import annotations

import time
from typing import Dict, List, Sequence

import numpy as np

from . import binding, synth


def quality(labels, truth, k: int) -> Dict[str, float]:
    """Acc, macro F1 (classes matched to clusters one-to-one, maximising the matched count),
    NMI and ARI of predicted `labels` against `truth` (both in [0, k))."""
    from scipy.optimize import linear_sum_assignment
    from sklearn.metrics import adjusted_rand_score, normalized_mutual_info_score
    labels = np.asarray(labels, dtype=np.int64)
    truth = np.asarray(truth, dtype=np.int64)
    C = np.zeros((k, k), dtype=np.int64)          # C[cluster, class]
    np.add.at(C, (labels, truth), 1)
    r, c = linear_sum_assignment(-C)
    matched = C[r, c]
    acc = matched.sum() / labels.shape[0]
    size_pred = C.sum(axis=1)[r]
    size_true = C.sum(axis=0)[c]
    with np.errstate(divide="ignore", invalid="ignore"):
        prec = np.where(size_pred > 0, matched / size_pred, 0.0)
        rec = np.where(size_true > 0, matched / size_true, 0.0)
        f1 = np.where(prec + rec > 0, 2 * prec * rec / (prec + rec), 0.0)
    # classes left without a cluster (k x k matching covers all) count as F1 0 through the mean
    return {"acc": float(acc), "f1": float(f1.sum() / k),
            "nmi": float(normalized_mutual_info_score(truth, labels)),
            "ari": float(adjusted_rand_score(truth, labels))}


def hard_graph(n: int = 100_000, k: int = 20, intra: float = 0.4, sep: float = 0.45, seed: int = 7000):
    """A planted-partition graph with weak signals on both sides (for the study only): a power-law
    SBM of mean degree 20 and exponent 2.5 with a 40% intra-cluster edge fraction, and BF16
    attributes d = 128 from a Gaussian mixture whose centres are only `sep` apart in the units of
    the generator, so that neither the topology nor the KNN graph alone recovers the clusters
    and K, beta and gamma change the result."""
    rng = np.random.default_rng(seed)
    labels = synth.planted_labels(n, k, rng)
    p, i = synth.chung_lu_sbm(labels, k, 20.0, 2.5, intra, rng)
    cen = synth.gmm_centres(k, 128, sep, np.random.default_rng(seed + 1))
    X = synth.gmm_attributes(labels, cen, rng, "bf16")
    net = synth.Network(synth.GRAPH, n, k, X, "bf16", [p], [i], labels=labels,
                        name=f"hard graph n={n} k={k} mean-degree 20 intra {intra} gmm d=128 sep {sep} (bf16)")
    return net, synth.RunParams(K=10, knn_mode="bf16", q_dtype="f32")


def _workload(cfg, scale):
    if cfg == "hard":
        return hard_graph(n=max(2000, int(round(100_000 * scale))))
    return synth.make_config(cfg, scale=scale)


def _params(lib, net, prm, **over):
    p = dict(k=net.k, K=prm.K, alpha=prm.alpha, beta=prm.beta, gamma=prm.gamma, tau=prm.tau, T_i=prm.T_i,
             T_a=prm.T_a, eps_q=prm.eps_q, knn_mode=prm.knn_mode, q_dtype=prm.q_dtype)
    p.update(over)
    return lib.default_params(**p)


def run_once(lib, net, prm, **over) -> Dict:
    """One whole run (ancka_cluster) with parameters overridden; quality, conductance, timing."""
    import torch
    s, keep = lib.network(net)
    params = _params(lib, net, prm, **over)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    labels, info = lib.cluster(s, params)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    q = quality(labels.cpu().numpy(), net.labels, net.k)
    return {**q, "phi": info["best_phi"], "iterations": info["iterations"], "stop": info["stop_reason"],
            "ms": round(ms, 2), "knn_ms": round(info["phase_ms"]["knn"], 2)}


def sweep(lib, cfg: int, scale: float, param: str, values: Sequence, log=None) -> List[Dict]:
    """Quality, conductance and time of workload `cfg` (generated at `scale`) for each value of
    one parameter (K, beta, gamma, tau or alpha), the others at the workload's defaults."""
    net, prm = _workload(cfg, scale)
    out = []
    for v in values:
        r = run_once(lib, net, prm, **{param: v})
        r[param] = v
        out.append(r)
        if log:
            log(f"workload {cfg} n={net.n} {param}={v}: acc {r['acc']:.4f} nmi {r['nmi']:.4f} phi {r['phi']:.5f} "
                f"iters {r['iterations']} {r['ms']:.1f} ms")
    return out


def convergence_trace(lib, cfg: int, scale: float, T: int, start: str = "greedy", seed: int = 0,
                      log=None) -> List[Dict]:
    """phi_t and quality of the labels Discretize gives at every iteration t = 0 .. T with early
    termination off (Sec. 8.4): Q^(0) from the greedy initial BCM (Alg. 4) or from random
    labels (`start` = 'random'), then Q^(t) = qf(P Q^(t-1)), Discretize of Q^(t)[:, 1:] and its
    MHC at every t.  Row t = 0 scores the starting labels themselves."""
    import torch
    net, prm = _workload(cfg, scale)
    s, keep = lib.network(net)
    X = binding.upload_attributes(net.X, net.x_dtype)
    idx, sim, _ = lib.knn(X, prm.K, prm.knn_mode)
    op = lib.build_operator(s, idx, sim, prm.K, prm.beta, prm.q_dtype)
    del X, idx, sim
    k = net.k
    if start == "greedy":
        y0 = op.init_bcm(k, prm.alpha, prm.T_i)
    else:
        rng = np.random.default_rng(seed)
        y0 = torch.from_numpy(rng.integers(0, k, size=net.n).astype(np.int32)).cuda()
    Q = op.initial_block(k, labels=y0)
    rows = []
    phi0 = op.mhc(y0, k, prm.alpha, prm.gamma)
    rows.append({"t": 0, "phi": phi0, **quality(y0.cpu().numpy(), net.labels, k)})
    for t in range(1, T + 1):
        _, dq = op.orth_iter(Q, k + 1, 1)
        yt, _, _, _ = lib.discretize(Q[:, 1:], k, prm.disc_max_iter)
        phi = op.mhc(yt, k, prm.alpha, prm.gamma)
        rows.append({"t": t, "phi": phi, "dq": dq, **quality(yt.cpu().numpy(), net.labels, k)})
    if log:
        best = min(rows, key=lambda r: r["phi"])
        log(f"workload {cfg} n={net.n} {start} start: phi_0 {rows[0]['phi']:.5f} -> phi_{T} {rows[-1]['phi']:.5f}, "
            f"best phi {best['phi']:.5f} at t={best['t']} (acc {best['acc']:.4f})")
    return rows


DEFAULT_STUDY = {
    # workload: (scale, parameter values); the paper's ranges cut to what the library supports
    "K": [2, 5, 10, 20, 30, 50, 64],
    "beta": [0.0, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 1.0],
    "gamma": [1, 2, 3, 4, 5],
    "tau": [1, 2, 5, 10],
}
STUDY_WORKLOADS = {2: 0.3, 3: 0.1, 4: 0.1, "hard": 1.0}


def study(lib, workloads: Dict[int, float] = None, params: Dict[str, Sequence] = None, T: int = 60,
          log=None) -> Dict:
    """The whole study: every parameter sweep on every workload, then convergence traces from
    the greedy and the random start.  Returns a JSON-ready dict."""
    workloads = workloads or STUDY_WORKLOADS
    params = params or DEFAULT_STUDY
    res = {"workloads": {}, "quality": "against the planted labels (Acc, macro F1, NMI, ARI)"}
    for cfg, scale in workloads.items():
        net, _ = _workload(cfg, scale)
        w = {"name": net.name, "sweeps": {}, "convergence": {}}
        for p, vals in params.items():
            w["sweeps"][p] = sweep(lib, cfg, scale, p, [v for v in vals if p != "K" or v <= net.n - 1], log=log)
        for start in ("greedy", "random"):
            w["convergence"][start] = convergence_trace(lib, cfg, scale, T, start=start, log=log)
        res["workloads"][str(cfg)] = w
    return res
