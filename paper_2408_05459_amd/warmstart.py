"""Learned warm start: training data from the plain method, training, warm-started runs.

Every arithmetic step runs in libancka's kernels (KNN, operator, orthogonal iteration,
Discretize, feature aggregation, MLP forward/backward/Adam, target rotation).  This module
sequences those calls and does one piece of host bookkeeping per training graph: the
assignment of its clusters to the shared mixture centres (Hungarian method on k x k cosines
of cluster-mean attributes), which fixes the column order of the target.

Training graphs come from the warm-start family of ``synth.make_warm_graph`` (hypergraphs
whose attribute mixtures share one set of centres), generated on host worker processes while
the GPU processes the previous graph.
"""
from __future__ import annotations

import multiprocessing as mp
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
from scipy.optimize import linear_sum_assignment

from . import binding, synth

H1 = 256
H2 = 256


def params_for(lib: binding.Lib, k: int, prm: synth.RunParams, **over):
    kw = dict(k=k, K=prm.K, alpha=prm.alpha, beta=prm.beta, gamma=prm.gamma, tau=prm.tau, T_i=prm.T_i,
              T_a=prm.T_a, eps_q=prm.eps_q, knn_mode=prm.knn_mode, q_dtype=prm.q_dtype)
    kw.update(over)
    return lib.default_params(**kw)


def centre_assignment(X: np.ndarray, labels: np.ndarray, centres: np.ndarray) -> np.ndarray:
    """colmap[c] = centre matched to cluster c: the assignment maximising the summed cosine
    between the clusters' mean normalised attribute vectors and the centres."""
    k = centres.shape[0]
    X = np.asarray(X, dtype=np.float32)
    nr = np.linalg.norm(X, axis=1)
    Xn = X / np.where(nr > 0, nr, 1.0)[:, None]
    onehot = np.zeros((k, X.shape[0]), dtype=np.float32)
    onehot[labels, np.arange(X.shape[0])] = 1.0
    sums = onehot @ Xn
    mn = np.linalg.norm(sums, axis=1)
    C = centres / np.linalg.norm(centres, axis=1, keepdims=True)
    score = (sums / np.where(mn > 0, mn, 1.0)[:, None]) @ C.T.astype(np.float32)
    _, colmap = linear_sum_assignment(-score.astype(np.float64))
    return colmap.astype(np.int32)


@dataclass
class Example:
    U: object              # device float n x ldu
    T: object              # device float n x k
    n: int
    iters: int             # orthogonal iterations the plain method ran
    seed: int


def _gen(args):
    n, seed = args
    net, prm = synth.make_warm_graph(n, seed)
    return net, prm


def generate(n: int, seeds: List[int], workers: int = 0):
    """Yield (seed, net, prm) in seed order; with workers > 0, host processes generate ahead."""
    if workers <= 0:
        for s in seeds:
            net, prm = _gen((n, s))
            yield s, net, prm
        return
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        for s, (net, prm) in zip(seeds, pool.imap(_gen, [(n, s) for s in seeds])):
            yield s, net, prm


def plain_block(lib: binding.Lib, s, X, k: int, prm: synth.RunParams):
    """The plain method's final eigenblock: the method runs to its own termination (Eqs.
    tcond-1/tcond-2) from the greedy start, then the block of that iteration is rebuilt from the
    same start (both steps are deterministic) and discretized.  Returns (op, Q, labels, R, t)."""
    idx, sim, _ = lib.knn(X, prm.K, prm.knn_mode)
    op = lib.build_operator(s, idx, sim, prm.K, prm.beta, prm.q_dtype)
    del idx, sim
    _, info = lib.cluster(None, params_for(lib, k, prm), op=op)
    t = info["iterations"]
    y0 = op.init_bcm(k, prm.alpha, prm.T_i)
    Q = op.initial_block(k, labels=y0)
    if t > 0:
        op.orth_iter(Q, k + 1, t)
    labels, R, _, _ = lib.discretize(Q[:, 1:], k, max_iter=prm.disc_max_iter)
    return op, Q, labels, R, t


def make_examples(lib: binding.Lib, n: int, seeds: List[int], workers: int = 0, log=None) -> List[Example]:
    """Training examples (U, T) of the warm-start family, one per seed, kept on the device."""
    centres = synth.warm_centres()
    out = []
    t0 = time.perf_counter()
    for s_i, net, prm in generate(n, seeds, workers):
        s, keep = lib.network(net)
        X = keep[-1]
        op, Q, labels, R, t = plain_block(lib, s, X, net.k, prm)
        colmap = centre_assignment(net.X, labels.cpu().numpy(), centres)
        T = lib.ws_target(Q[:, 1:], net.k, R, colmap)
        U = lib.ws_features(op, X)
        out.append(Example(U=U, T=T, n=net.n, iters=t, seed=s_i))
        del op, Q, keep, X
        if log and (len(out) % 20 == 0 or len(out) == len(seeds)):
            log(f"  training graphs: {len(out)}/{len(seeds)} ({time.perf_counter() - t0:.1f}s)")
    return out


@dataclass
class TrainLog:
    epoch_loss: List[float] = field(default_factory=list)
    seconds: float = 0.0
    steps: int = 0


def train(lib: binding.Lib, examples: List[Example], d: int, k: int, epochs: int = 10, lr: float = 1e-3,
          seed: int = 0, log=None):
    """Adam on the mean squared error, one step per training graph, graphs in a seeded order
    per epoch.  Returns (model, TrainLog)."""
    import torch
    ws = binding.WarmStart(lib, d, H1, H2, k, seed=seed)
    rng = np.random.default_rng(seed)
    tl = TrainLog()
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(len(examples))
        tot = 0.0
        for i in order:
            ex = examples[i]
            Z = ws.forward(ex.U, keep_acts=True)
            tot += ws.backward(Z, ex.T)
            ws.step(lr)
            tl.steps += 1
        tl.epoch_loss.append(tot / len(examples))
        if log:
            log(f"  epoch {ep}: mean loss {tl.epoch_loss[-1]:.5f}")
    torch.cuda.synchronize()
    tl.seconds = time.perf_counter() - t0
    return ws, tl


def mean_loss(ws: binding.WarmStart, examples: List[Example]) -> float:
    """Loss of the current model over examples (forward + loss only)."""
    tot = 0.0
    for ex in examples:
        Z = ws.forward(ex.U, keep_acts=True)
        tot += ws.backward(Z, ex.T)
    return tot / len(examples)


def run(lib: binding.Lib, s, X, k: int, prm: synth.RunParams, ws: Optional[binding.WarmStart] = None, **over):
    """One run of the method on an uploaded network, cold (ws None) or warm-started.

    Both runs build the KNN graph and the operator once; the warm run then aggregates the
    features with the operator's walk, evaluates the MLP and hands its block to the loop
    (which keeps the greedy start if that has the lower conductance).  `over` overrides run
    parameters (e.g. T_a).  Returns (labels, info, timings_ms)."""
    import torch
    tm = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx, sim, _ = lib.knn(X, prm.K, prm.knn_mode)
    torch.cuda.synchronize()
    tm["knn"] = (time.perf_counter() - t0) * 1e3
    t1 = time.perf_counter()
    op = lib.build_operator(s, idx, sim, prm.K, prm.beta, prm.q_dtype)
    tm["operator"] = (time.perf_counter() - t1) * 1e3
    zwarm = None
    if ws is not None:
        t2 = time.perf_counter()
        U = lib.ws_features(op, X)
        zwarm = ws.forward(U)
        torch.cuda.synchronize()
        tm["features_mlp"] = (time.perf_counter() - t2) * 1e3
        del U
    t3 = time.perf_counter()
    labels, info = lib.cluster(None, params_for(lib, k, prm, **over), zwarm=zwarm, op=op)
    tm["loop"] = (time.perf_counter() - t3) * 1e3
    tm["total"] = (time.perf_counter() - t0) * 1e3
    return labels, info, tm


def time_to_reach(info: dict, target_phi: float) -> Optional[int]:
    """First checked iteration t whose conductance is within target_phi (None if never)."""
    for t, phi in info["trace"]:
        if phi <= target_phi:
            return t
    return None
