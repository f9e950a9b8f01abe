"""Seeded synthetic attributed networks (planted partitions).

This module only draws inputs: labels, topologies and attribute matrices.  It
holds none of the clustering method's arithmetic, and it is the one module that
both the FP64 oracle tests and the GPU path take their inputs from.

The paper evaluates on real attributed hypergraphs, graphs and multiplex graphs
(Sec. 8.1, dataset table); none of them is available here, so planted-partition
networks of the same three kinds stand in for them.  Distribution choices:

* planted labels: a seeded permutation of 0..n-1 taken mod k, so the node index
  order carries no cluster information;
* hyperedges: a home cluster drawn uniformly, each member drawn from the home
  cluster with probability ``intra`` and otherwise uniformly from the other
  clusters; repeated members are redrawn; sizes are uniform or truncated Zipf;
* graphs / multiplex layers: Chung-Lu stochastic block model.  Node weights
  follow a Pareto law with density proportional to theta^-exponent, lower end
  mean*(exponent-2)/(exponent-1), capped at sqrt(n*mean) and rescaled to the
  target mean; an edge picks u proportionally to theta, then v proportionally
  to theta inside u's cluster with probability ``intra`` and outside it
  otherwise; self loops are dropped, duplicates merged, both directions stored;
* dense attributes: Gaussian mixture with unit noise and centres drawn
  N(0, (c^2/2) I_d), so that centres sit about c*sqrt(d) apart;
* binary attributes: attribute j belongs to cluster j mod k and is set with a
  three times higher rate inside the node's own block.

BF16 attribute matrices are returned as float32 arrays whose values are exactly
representable in bfloat16 (rounded to nearest even).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

HYPERGRAPH, GRAPH, MULTIPLEX = 0, 1, 2


@dataclasses.dataclass
class Network:
    kind: int                      # HYPERGRAPH / GRAPH / MULTIPLEX
    n: int
    k: int
    X: np.ndarray                  # n x d attributes (float64, float32 or bf16-valued float32)
    x_dtype: str                   # "f64", "f32" or "bf16"
    ptrs: List[np.ndarray]         # hypergraph: [he_ptr (m+1)]; graph/multiplex: one CSR row pointer per layer
    idxs: List[np.ndarray]         # matching int32 index arrays
    m: int = 0                     # number of hyperedges (hypergraph only)
    labels: Optional[np.ndarray] = None   # planted labels (ground truth, not an input of the method)
    name: str = ""

    @property
    def d(self) -> int:
        return int(self.X.shape[1])

    @property
    def L(self) -> int:
        return len(self.ptrs)


@dataclasses.dataclass
class RunParams:
    K: int = 10
    alpha: float = 0.2
    beta: float = 0.5
    gamma: int = 3
    tau: int = 5
    T_i: int = 25
    T_a: int = 1000
    eps_q: float = 0.005
    disc_max_iter: int = 30
    knn_mode: str = "f32"          # "f64", "f32" or "bf16"
    q_dtype: str = "f32"           # "f64" or "f32"


def round_to_bf16(a: np.ndarray) -> np.ndarray:
    """Round finite float32 values to the nearest bfloat16 (ties to even); returns float32.
    (For finite inputs the 32-bit sum below cannot overflow.)"""
    a = np.array(a, dtype=np.float32, copy=True, order="C")
    b = a.view(np.uint32)
    lsb = (b >> np.uint32(16)) & np.uint32(1)
    b += np.uint32(0x7FFF)
    b += lsb
    b &= np.uint32(0xFFFF0000)
    return a


def planted_labels(n: int, k: int, rng: np.random.Generator) -> np.ndarray:
    return (rng.permutation(n) % k).astype(np.int32)


def _cluster_index(labels: np.ndarray, k: int):
    order = np.argsort(labels, kind="stable").astype(np.int64)
    sizes = np.bincount(labels, minlength=k).astype(np.int64)
    start = np.zeros(k + 1, dtype=np.int64)
    start[1:] = np.cumsum(sizes)
    return order, sizes, start


def truncated_zipf_sizes(count: int, lo: int, hi: int, s: float, rng) -> np.ndarray:
    vals = np.arange(lo, hi + 1, dtype=np.int64)
    p = vals.astype(np.float64) ** (-s)
    p /= p.sum()
    return rng.choice(vals, size=count, p=p)


def hypergraph_incidence(labels: np.ndarray, k: int, sizes: np.ndarray, intra: float,
                         rng: np.random.Generator):
    """Hyperedge -> member lists (CSR over hyperedges), members distinct."""
    n = labels.shape[0]
    m = sizes.shape[0]
    order, csize, start = _cluster_index(labels, k)
    home = rng.integers(0, k, size=m)
    he_ptr = np.zeros(m + 1, dtype=np.int64)
    he_ptr[1:] = np.cumsum(sizes)
    nnz = int(he_ptr[-1])
    edge_of = np.repeat(np.arange(m, dtype=np.int64), sizes)

    def draw(which: np.ndarray) -> np.ndarray:
        c = home[edge_of[which]]
        inside = rng.random(which.shape[0]) < intra
        u = rng.random(which.shape[0])
        out = np.empty(which.shape[0], dtype=np.int64)
        ci = c[inside]
        out[inside] = order[start[ci] + np.minimum((u[inside] * csize[ci]).astype(np.int64), csize[ci] - 1)]
        co = c[~inside]
        rest = n - csize[co]
        pos = np.minimum((u[~inside] * rest).astype(np.int64), rest - 1)
        pos = np.where(pos >= start[co], pos + csize[co], pos)
        out[~inside] = order[pos]
        return out

    members = draw(np.arange(nnz, dtype=np.int64))
    for _ in range(1000):
        key = edge_of * n + members
        srt = np.argsort(key, kind="stable")
        ks = key[srt]
        dup = np.zeros(nnz, dtype=bool)
        dup[srt[1:][ks[1:] == ks[:-1]]] = True
        if not dup.any():
            break
        which = np.nonzero(dup)[0]
        members[which] = draw(which)
    return he_ptr, members.astype(np.int32)


def chung_lu_weights(n: int, mean: float, exponent: float, rng) -> np.ndarray:
    tmin = mean * (exponent - 2.0) / (exponent - 1.0)
    theta = tmin * rng.random(n) ** (-1.0 / (exponent - 1.0))
    theta = np.minimum(theta, math.sqrt(n * mean))
    return theta * (mean / theta.mean())


def _draw_proportional(count: int, nodes: np.ndarray, weights: np.ndarray, rng) -> np.ndarray:
    """`count` i.i.d. draws from `nodes` with probability proportional to `weights`, in random
    order (multinomial counts per node, expanded and shuffled)."""
    if count == 0:
        return np.empty(0, dtype=np.int64)
    p = weights / weights.sum()
    p[-1] = max(0.0, 1.0 - p[:-1].sum())
    c = rng.multinomial(count, p)
    out = np.repeat(nodes.astype(np.int64), c)
    rng.shuffle(out)
    return out


def chung_lu_sbm(labels: np.ndarray, k: int, mean: float, exponent: float, intra: float,
                 rng: np.random.Generator):
    """Undirected planted-partition Chung-Lu graph, returned as a symmetric CSR."""
    n = labels.shape[0]
    theta = chung_lu_weights(n, mean, exponent, rng)
    order, csize, start = _cluster_index(labels, k)
    E = int(round(n * mean / 2.0))
    allnodes = np.arange(n, dtype=np.int64)

    u = _draw_proportional(E, allnodes, theta, rng)
    lu = labels[u]
    inside = rng.random(E) < intra
    v = np.empty(E, dtype=np.int64)
    # intra-cluster partner: proportional to theta inside u's cluster
    sel = np.nonzero(inside)[0]
    grp = np.argsort(lu[sel], kind="stable")
    sel = sel[grp]
    cnt = np.bincount(lu[sel], minlength=k)
    off = 0
    for c in range(k):
        members = order[start[c]:start[c + 1]]
        v[sel[off:off + cnt[c]]] = _draw_proportional(int(cnt[c]), members, theta[members], rng)
        off += cnt[c]
    # inter-cluster partner: proportional to theta over all nodes, redrawn while it falls in
    # u's own cluster (rejection)
    todo = np.nonzero(~inside)[0]
    while todo.shape[0] > 0:
        cand = _draw_proportional(todo.shape[0], allnodes, theta, rng)
        ok = labels[cand] != lu[todo]
        v[todo[ok]] = cand[ok]
        todo = todo[~ok]
    keep = u != v
    a = np.minimum(u[keep], v[keep])
    b = np.maximum(u[keep], v[keep])
    key = np.unique(a * n + b)
    a = key // n
    b = key % n
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    key = np.sort(rows * n + cols)
    rows = key // n
    cols = (key % n).astype(np.int32)
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=ptr[1:])
    return ptr, cols


def gmm_centres(k: int, d: int, c: float, rng) -> np.ndarray:
    return rng.standard_normal((k, d)) * math.sqrt(c * c / 2.0)


def gmm_attributes(labels: np.ndarray, centres: np.ndarray, rng, out_dtype: str) -> np.ndarray:
    n = labels.shape[0]
    d = centres.shape[1]
    X = np.empty((n, d), dtype=np.float32)
    cen = centres.astype(np.float32)
    blk = 1 << 16
    for s in range(0, n, blk):
        e = min(n, s + blk)
        rng.standard_normal((e - s, d), dtype=np.float32, out=X[s:e])
        X[s:e] += cen[labels[s:e]]
        if out_dtype == "bf16":
            X[s:e] = round_to_bf16(X[s:e])
    if out_dtype == "f64":
        X = X.astype(np.float64)
    return X


def binary_attributes(labels: np.ndarray, k: int, d: int, density: float, ratio: float, rng) -> np.ndarray:
    n = labels.shape[0]
    p = density * k / (k + ratio - 1.0)
    own = (np.arange(d)[None, :] % k) == labels[:, None]
    rate = np.where(own, ratio * p, p)
    return (rng.random((n, d)) < rate).astype(np.float64)


# ----------------------------------------------------------------------------------------
# The five workloads.  ``scale`` shrinks n (and m) keeping every distribution, which gives
# parity-sized variants of the large ones.

def make_config(cfg: int, scale: float = 1.0, seed: Optional[int] = None):
    """Return (Network, RunParams) for workload ``cfg`` in 1..5."""
    if seed is None:
        seed = 1000 * cfg
    rng = np.random.default_rng(seed)
    if cfg == 1:
        n = max(40, int(round(2000 * scale)))
        k = 6
        labels = planted_labels(n, k, rng)
        m = max(10, int(round(1500 * scale)))
        sizes = rng.integers(2, 11, size=m)
        he_ptr, he_idx = hypergraph_incidence(labels, k, sizes, 0.8, rng)
        X = binary_attributes(labels, k, 500, 0.02, 3.0, rng)
        net = Network(HYPERGRAPH, n, k, X, "f64", [he_ptr], [he_idx], m=m, labels=labels,
                      name=f"hypergraph n={n} k={k} m={m} binary d=500 (f64)")
        return net, RunParams(K=10, knn_mode="f64", q_dtype="f64")
    if cfg == 2:
        n = max(100, int(round(100_000 * scale)))
        k = 20
        labels = planted_labels(n, k, rng)
        m = max(20, int(round(200_000 * scale)))
        sizes = truncated_zipf_sizes(m, 2, min(50, n // k), 2.0, rng)
        he_ptr, he_idx = hypergraph_incidence(labels, k, sizes, 0.7, rng)
        cen = gmm_centres(k, 1000, 2.0, np.random.default_rng(seed + 1))
        X = gmm_attributes(labels, cen, rng, "f32")
        net = Network(HYPERGRAPH, n, k, X, "f32", [he_ptr], [he_idx], m=m, labels=labels,
                      name=f"hypergraph n={n} k={k} m={m} gmm d=1000 (f32)")
        return net, RunParams(K=10, knn_mode="f32", q_dtype="f32")
    if cfg == 3:
        n = max(200, int(round(500_000 * scale)))
        k = 10
        labels = planted_labels(n, k, rng)
        ptrs, idxs = [], []
        for intra in (0.6, 0.7, 0.8):
            p, i = chung_lu_sbm(labels, k, 20.0, 2.5, intra, rng)
            ptrs.append(p)
            idxs.append(i)
        cen = gmm_centres(k, 256, 2.0, np.random.default_rng(seed + 1))
        X = gmm_attributes(labels, cen, rng, "bf16")
        net = Network(MULTIPLEX, n, k, X, "bf16", ptrs, idxs, labels=labels,
                      name=f"multiplex L=3 n={n} k={k} mean-degree 20 gmm d=256 (bf16)")
        return net, RunParams(K=10, knn_mode="bf16", q_dtype="f32")
    if cfg == 4:
        n = max(500, int(round(2_500_000 * scale)))
        k = 50
        labels = planted_labels(n, k, rng)
        p, i = chung_lu_sbm(labels, k, 30.0, 2.2, 0.65, rng)
        cen = gmm_centres(k, 128, 1.5, np.random.default_rng(seed + 1))
        X = gmm_attributes(labels, cen, rng, "bf16")
        net = Network(GRAPH, n, k, X, "bf16", [p], [i], labels=labels,
                      name=f"graph n={n} k={k} mean-degree 30 gmm d=128 (bf16)")
        return net, RunParams(K=10, knn_mode="bf16", q_dtype="f32")
    if cfg == 5:
        return make_warm_graph(n=max(300, int(round(1_000_000 * scale))), seed=5000 if seed == 5000 else seed)
    raise ValueError(f"unknown workload {cfg}")


WARM_CENTRE_SEED = 5999


def warm_centres(k: int = 30, d: int = 512) -> np.ndarray:
    """Mixture centres shared by every graph of the warm-start family."""
    return gmm_centres(k, d, 2.0, np.random.default_rng(WARM_CENTRE_SEED))


def make_warm_graph(n: int, seed: int, k: int = 30, d: int = 512, mean_deg: float = 25.0):
    """Hypergraph family of the learned warm start (shared GMM centres)."""
    rng = np.random.default_rng(seed)
    labels = planted_labels(n, k, rng)
    mean_size = 5.5975
    m = max(k, int(round(n * mean_deg / mean_size)))
    sizes = truncated_zipf_sizes(m, 2, min(50, max(2, n // k)), 2.0, rng)
    he_ptr, he_idx = hypergraph_incidence(labels, k, sizes, 0.7, rng)
    cen = warm_centres(k, d)
    X = gmm_attributes(labels, cen, rng, "bf16")
    net = Network(HYPERGRAPH, n, k, X, "bf16", [he_ptr], [he_idx], m=m, labels=labels,
                  name=f"hypergraph n={n} k={k} m={m} gmm d={d} (bf16)")
    return net, RunParams(K=10, knn_mode="bf16", q_dtype="f32")


def describe(net: Network) -> dict:
    """Realised statistics of a generated network (for logs)."""
    out = {"name": net.name, "n": net.n, "k": net.k, "d": net.d}
    if net.kind == HYPERGRAPH:
        deg = np.bincount(net.idxs[0], minlength=net.n)
        lab = net.labels
        ptr = net.ptrs[0]
        out.update(m=net.m, nnz=int(ptr[-1]), mean_node_degree=float(deg.mean()),
                   isolated=int((deg == 0).sum()))
        if lab is not None:
            home = []
            for e in range(min(net.m, 2000)):
                mem = net.idxs[0][ptr[e]:ptr[e + 1]]
                home.append(np.bincount(lab[mem], minlength=net.k).max() / len(mem))
            out["mean_majority_fraction"] = float(np.mean(home))
    else:
        for l in range(net.L):
            ptr, idx = net.ptrs[l], net.idxs[l]
            deg = np.diff(ptr)
            rows = np.repeat(np.arange(net.n), deg)
            intra = float((net.labels[rows] == net.labels[idx]).mean()) if net.labels is not None else None
            out[f"layer{l}"] = dict(nnz=int(ptr[-1]), mean_degree=float(deg.mean()),
                                    max_degree=int(deg.max()), isolated=int((deg == 0).sum()),
                                    intra_fraction=intra)
    zero_rows = int((np.abs(net.X).sum(1) == 0).sum())
    out["zero_attribute_rows"] = zero_rows
    return out
