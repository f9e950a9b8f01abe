"""FP64 oracle of the clustering path (TEST INFRASTRUCTURE ONLY; see package docstring).

Plain numpy / scipy.sparse in float64.  Library primitives used as single steps:
matrix products (dense and sparse), numpy.linalg.qr (Householder QR),
numpy.linalg.svd.  No blocking, fusion or reordering beyond what the paper's
equations state.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

HYPERGRAPH, GRAPH, MULTIPLEX = 0, 1, 2

__all__ = [
    "HYPERGRAPH", "GRAPH", "MULTIPLEX", "normalize_rows", "cosine_rows", "knn", "knn_adjacency",
    "topology_transition", "betas", "Operator", "build_operator", "apply_P", "transition_dense",
    "centres", "init_bcm", "normalized_bcm", "fill_vector", "initial_q", "qr_pos", "orth_iter",
    "discretize", "complete_null", "mhc", "ClusterReport", "cluster", "multi_hop_dense",
]


# --------------------------------------------------------------------------------------
# Attribute prologue and KNN graph (Sec. 3.1; Alg. 6, normalisation step)

def normalize_rows(X):
    """x_i / ||x_i||_2; rows with zero norm stay zero and are flagged (Alg. 6, normalisation step).

    Reading: a zero attribute vector has no cosine similarity to anything, so it is never a
    neighbour candidate and has no neighbours (its beta_i is 0 by Eq. beta_i)."""
    X = np.asarray(X, dtype=np.float64)
    nrm = np.sqrt((X * X).sum(axis=1))
    zero = nrm == 0.0
    Xh = np.zeros_like(X)
    Xh[~zero] = X[~zero] / nrm[~zero, None]
    return Xh, zero


def cosine_rows(X, rows, sq=None, cols=None):
    """f(v_i, v_j) = cosine(X[i], X[j]) for i in ``rows`` and j in ``cols`` (a range c0..c1-1,
    default all nodes) (Sec. 3.1).

    Computed as (x_i . x_j) / sqrt(||x_i||^2 ||x_j||^2) in FP64.  Self pairs and zero rows
    are set to -inf (self is excluded from the K nearest neighbours, Sec. 3.1).  ``sq``, the
    squared row norms, may be passed in when the caller already holds them."""
    X = np.asarray(X, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    if sq is None:
        sq = (X * X).sum(axis=1)
    c0, c1 = (0, X.shape[0]) if cols is None else cols
    S = X[rows] @ X[c0:c1].T
    with np.errstate(divide="ignore", invalid="ignore"):
        S /= np.sqrt(sq[rows][:, None] * sq[None, c0:c1])
    S[:, sq[c0:c1] == 0.0] = -np.inf
    S[sq[rows] == 0.0, :] = -np.inf
    own = (rows >= c0) & (rows < c1)
    S[np.nonzero(own)[0], rows[own] - c0] = -np.inf
    return S


def knn(X, K, rows=None, block=512, width=16384, threads=None):
    """N_K(v_i): the K nodes other than v_i with the largest cosine similarity (Sec. 3.1).

    Ties are broken by the smaller node index, i.e. candidates are ordered by the key
    (-f, j).  A zero query row, or a row with fewer than K valid candidates, is padded with
    index -1 and similarity 0.  Returns (idx int64 [r, K], sim float64 [r, K]) sorted by key.

    For each query row: t0, the K-th largest valid similarity among the first ``width``
    nodes (-inf when there are fewer than K of them).  The row holds at least K valid
    similarities >= t0, so its K-th largest is >= t0 and every member of its top K by the
    key is among the valid entries >= t0.  Those entries are collected slice by slice of
    ``width`` columns (on ``threads`` threads, each with single-threaded BLAS), ordered by
    (-f, j), and the first K kept (all of them when there are fewer than K).  Within a slice
    the cosine formula is evaluated only where the dot product passes a bound that no entry
    >= t0 can fail."""
    from threadpoolctl import threadpool_limits

    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows, dtype=np.int64)
    sq = (X * X).sum(axis=1)
    nrm = np.sqrt(sq)
    out_i = np.full((rows.shape[0], K), -1, dtype=np.int64)
    out_s = np.zeros((rows.shape[0], K), dtype=np.float64)
    w0 = min(n, width)
    slices = [(c0, min(n, c0 + width)) for c0 in range(0, n, width)]
    with threadpool_limits(limits=1, user_api="blas"), \
            ThreadPoolExecutor(max_workers=threads or os.cpu_count() or 1) as ex:
        for b0 in range(0, rows.shape[0], block):
            rb = rows[b0:b0 + block]
            S0 = cosine_rows(X, rb, sq, (0, w0))
            t0 = np.full(rb.shape[0], -np.inf)
            if w0 >= K:
                kth = np.partition(S0, w0 - K, axis=1)[:, w0 - K]   # -inf sorts lowest
                t0 = np.where(kth > -np.inf, kth, -np.inf)

            def survivors(c):
                # entries whose cosine can reach t0: dot >= (t0 - 1e-12) |x_i| |x_j| (the
                # margin exceeds the rounding of both sides by far); their cosines are then
                # computed by the formula above, and self pairs and zero rows dropped
                c0, c1 = c
                # (t0 = -inf against a zero norm gives NaN, which passes nothing: zero rows
                # are never candidates)
                D = X[rb] @ X[c0:c1].T
                with np.errstate(divide="ignore", invalid="ignore"):
                    r, j = np.nonzero(D >= ((t0 - 1e-12) * nrm[rb])[:, None] * nrm[None, c0:c1])
                    jj = j + c0
                    f = D[r, j] / np.sqrt(sq[rb[r]] * sq[jj])
                ok = (sq[rb[r]] > 0.0) & (sq[jj] > 0.0) & (rb[r] != jj) & (f >= t0[r])
                return r[ok], jj[ok], f[ok]

            parts = list(ex.map(survivors, slices))
            r = np.concatenate([p[0] for p in parts])
            j = np.concatenate([p[1] for p in parts])
            s = np.concatenate([p[2] for p in parts])
            order = np.lexsort((j, -s, r))
            r, j, s = r[order], j[order], s[order]
            pos = np.arange(r.shape[0]) - np.searchsorted(r, r)
            keep = pos < K
            out_i[b0 + r[keep], pos[keep]] = j[keep]
            out_s[b0 + r[keep], pos[keep]] = s[keep]
    return out_i, out_s


def knn_adjacency(n, nbr_idx, nbr_sim):
    """A_K of Eq. (AK): 0 if neither is the other's neighbour, 2f if mutual, f if one-way.

    This equals W + W^T with W[i, j] = f(i, j) for j in N_K(i).  Reading for dense real
    attributes: edges whose cosine is <= 0 are dropped from W, since the walk of Definition 1
    needs non-negative transition weights."""
    nbr_idx = np.asarray(nbr_idx, dtype=np.int64)
    nbr_sim = np.asarray(nbr_sim, dtype=np.float64)
    r = np.repeat(np.arange(nbr_idx.shape[0]), nbr_idx.shape[1])
    c = nbr_idx.reshape(-1)
    v = nbr_sim.reshape(-1)
    keep = (c >= 0) & (v > 0.0)
    W = sp.csr_matrix((v[keep], (r[keep], c[keep])), shape=(n, n))
    return (W + W.T).tocsr()


# --------------------------------------------------------------------------------------
# Topology transition matrices P_N (Sec. 6.1: Eqs. rw-hg, rw-ag, rw-mg)

def _binary(M):
    M = M.tocsr()
    M.sum_duplicates()
    M.data[:] = 1.0
    M.eliminate_zeros()
    return M


def _sym_adjacency(n, ptr, idx):
    """Undirected simple adjacency: a reversed edge is added for each directed edge
    (Sec. 6.1, attributed graph), duplicates merged (A is binary, Sec. 2), self loops
    dropped."""
    ptr = np.asarray(ptr, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    rows = np.repeat(np.arange(n), np.diff(ptr))
    A = sp.csr_matrix((np.ones(idx.shape[0]), (rows, idx)), shape=(n, n))
    A = _binary(A + A.T)
    A.setdiag(0.0)
    A.eliminate_zeros()
    return A


def _diag_inv(v):
    out = np.zeros_like(v, dtype=np.float64)
    nz = v != 0
    out[nz] = 1.0 / v[nz]
    return sp.diags(out)


def topology_transition(kind, n, ptrs, idxs, m=0, literal_rw_mg=False):
    """P_N and the node degree delta(v) for the three network kinds.

    * hypergraph (Eq. rw-hg): P_N = P_V P_E with P_V = D_V^-1 H^T, P_E = D_E^-1 H; H is the
      binary m x n incidence (repeated members merged; an empty hyperedge is rejected);
      delta(v) = number of incident hyperedges.
    * graph (Eq. rw-ag): P_N = D^-1 A after symmetrisation; delta = degree.
    * multiplex (Eq. rw-mg): average of the layer walks D_l^-1 A_l.  Reading for a node
      without edges in some layers: the average runs over the L_i layers where it has
      edges, so its row stays stochastic (``literal_rw_mg`` uses 1/L instead).
      delta = degree summed over layers (Sec. 6.2, centre ranking).
    Returns a dict with P_N (csr) and delta, plus P_V, P_E for hypergraphs."""
    if kind == HYPERGRAPH:
        he_ptr = np.asarray(ptrs[0], dtype=np.int64)
        he_idx = np.asarray(idxs[0], dtype=np.int64)
        sizes = np.diff(he_ptr)
        if (sizes <= 0).any():
            raise ValueError("empty hyperedge")
        er = np.repeat(np.arange(m), sizes)
        H = _binary(sp.csr_matrix((np.ones(he_idx.shape[0]), (er, he_idx)), shape=(m, n)))
        delta = np.asarray(H.sum(axis=0)).ravel()
        esize = np.asarray(H.sum(axis=1)).ravel()
        P_V = (_diag_inv(delta) @ H.T).tocsr()
        P_E = (_diag_inv(esize) @ H).tocsr()
        return {"P_N": (P_V @ P_E).tocsr(), "P_V": P_V, "P_E": P_E, "delta": delta}
    if kind == GRAPH:
        A = _sym_adjacency(n, ptrs[0], idxs[0])
        deg = np.asarray(A.sum(axis=1)).ravel()
        return {"P_N": (_diag_inv(deg) @ A).tocsr(), "delta": deg}
    if kind == MULTIPLEX:
        layers = [_sym_adjacency(n, p, i) for p, i in zip(ptrs, idxs)]
        degs = [np.asarray(A.sum(axis=1)).ravel() for A in layers]
        L = len(layers)
        active = sum((d > 0).astype(np.float64) for d in degs)
        P = sp.csr_matrix((n, n))
        for A, d in zip(layers, degs):
            w = np.zeros(n)
            nz = d > 0
            if literal_rw_mg:
                w[nz] = 1.0 / (L * d[nz])
            else:
                w[nz] = 1.0 / (active[nz] * d[nz])
            P = P + sp.diags(w) @ A
        return {"P_N": P.tocsr(), "delta": sum(degs)}
    raise ValueError(kind)


def betas(zero, delta, D_K, beta):
    """beta_i of Eq. (beta_i): 0 for a zero attribute vector, else 1 if delta(v_i) = 0,
    else beta.  Reading: a node whose KNN row is empty (every similarity dropped) also gets
    beta_i = 0, since the walk has no KNN edge to follow."""
    zero = np.asarray(zero, dtype=bool)
    delta = np.asarray(delta)
    D_K = np.asarray(D_K)
    b = np.where(delta == 0, 1.0, float(beta))
    b[zero | (D_K == 0)] = 0.0
    return b


@dataclass
class Operator:
    kind: int
    n: int
    P_N: sp.csr_matrix
    P_K: sp.csr_matrix
    beta: np.ndarray
    selfloop: np.ndarray
    delta: np.ndarray
    P_V: Optional[sp.csr_matrix] = None
    P_E: Optional[sp.csr_matrix] = None


def build_operator(kind, n, ptrs, idxs, m, zero, nbr_idx, nbr_sim, beta, literal_rw_mg=False,
                   literal_zero_rows=False):
    """Assemble P = (I - B) P_N + B P_K (Eq. p-mat-ancka) without multiplying it out.

    P_K = D_K^-1 A_K (Alg. 6, graph construction).  Reading for a node whose row of P would be empty
    (beta_i = 0 and no topology edge): it gets a self loop P[i, i] = 1 so that P stays
    row-stochastic (switch off with ``literal_zero_rows``)."""
    top = topology_transition(kind, n, ptrs, idxs, m, literal_rw_mg)
    A_K = knn_adjacency(n, nbr_idx, nbr_sim)
    D_K = np.asarray(A_K.sum(axis=1)).ravel()
    P_K = (_diag_inv(D_K) @ A_K).tocsr()
    b = betas(zero, top["delta"], D_K, beta)
    selfloop = (b == 0.0) & (top["delta"] == 0)
    if literal_zero_rows:
        selfloop[:] = False
    return Operator(kind, n, top["P_N"], P_K, b, selfloop, top["delta"], top.get("P_V"), top.get("P_E"))


def apply_P(op: Operator, Q):
    """Z = (I - B) P_N Q + B P_K Q (Eqs. zt and p-mat-ancka); for hypergraphs P_N Q is
    evaluated as P_V (P_E Q) so that P_V P_E is never formed (Eq. zt)."""
    Q = np.asarray(Q, dtype=np.float64)
    if op.kind == HYPERGRAPH:
        PNQ = op.P_V @ (op.P_E @ Q)
    else:
        PNQ = op.P_N @ Q
    b = op.beta[:, None] if Q.ndim == 2 else op.beta
    Z = (1.0 - b) * PNQ + b * (op.P_K @ Q)
    if op.selfloop.any():
        Z[op.selfloop] += Q[op.selfloop]
    return Z


def transition_dense(op: Operator):
    """P as a dense n x n matrix (tiny inputs only)."""
    return apply_P(op, np.eye(op.n))


def multi_hop_dense(op: Operator, alpha, gamma):
    """S = alpha * sum_{l=0..gamma} (1-alpha)^l P^l (Eq. approx-multi-hop), dense."""
    P = transition_dense(op)
    S = np.zeros_like(P)
    Pl = np.eye(op.n)
    for l in range(gamma + 1):
        S += alpha * (1.0 - alpha) ** l * Pl
        Pl = Pl @ P
    return S


# --------------------------------------------------------------------------------------
# Greedy initialisation (Alg. 3 / Alg. 4, greedy start, Eqs. pi_c_t and argmaxlabel)

def centres(delta, k):
    """V_c: the k nodes of largest degree, listed by node index (Alg. 4, choice of the centres).
    Reading for degree ties: the smaller index ranks first."""
    delta = np.asarray(delta)
    order = np.lexsort((np.arange(delta.shape[0]), -delta))
    return np.sort(order[:k])


def init_bcm(op: Operator, k, alpha, T_i):
    """Pi^(t) = (1-alpha) Pi^(t-1) P_N + alpha Z_0 for T_i steps, then the label of v_j is
    argmax_l Pi[l, j] (the smallest l on ties, so an all-zero column gives label 0)."""
    Vc = centres(op.delta, k)
    n = op.n
    Z0 = np.zeros((k, n))
    Z0[np.arange(k), Vc] = 1.0
    Pi = alpha * Z0
    for _ in range(T_i):
        if op.kind == HYPERGRAPH:
            PiPN = (op.P_V.T @ Pi.T).T            # Pi P_V
            PiPN = (op.P_E.T @ PiPN.T).T          # (Pi P_V) P_E
        else:
            PiPN = (op.P_N.T @ Pi.T).T
        Pi = (1.0 - alpha) * PiPN + alpha * Z0
    return np.argmax(Pi, axis=0).astype(np.int64), Pi


def normalized_bcm(labels, k):
    """h(Y) = (Y^T Y)^(-1/2) Y (Eq. norm-y); an empty cluster gives a zero column."""
    labels = np.asarray(labels, dtype=np.int64)
    n = labels.shape[0]
    cnt = np.bincount(labels, minlength=k).astype(np.float64)
    Yh = np.zeros((n, k))
    Yh[np.arange(n), labels] = 1.0 / np.sqrt(cnt[labels])
    return Yh


def fill_vector(n, j):
    """Deterministic replacement for a dependent column j: cos(pi (i + 1/2) j / n)."""
    i = np.arange(n, dtype=np.float64)
    return np.cos(math.pi * (i + 0.5) * j / n)


def initial_q(C, tol=1e-8):
    """Orthonormal basis of the starting block (Alg. 4, starting block).

    Reading: [1/sqrt(n) 1 | h(Y0)] has rank k at most, because the all-ones vector is the
    sum of the cluster indicators; it is orthonormalised column by column (Gram-Schmidt,
    applied twice), and a column whose residual is below ``tol`` times its norm, or a zero
    column, is replaced by fill_vector(n, j) before orthonormalising it."""
    C = np.asarray(C, dtype=np.float64)
    n, p = C.shape
    Q = np.zeros((n, p))
    for j in range(p):
        v = C[:, j].copy()
        nv = np.linalg.norm(v)
        ok = False
        if nv > 0.0:
            w = v - Q[:, :j] @ (Q[:, :j].T @ v)
            w = w - Q[:, :j] @ (Q[:, :j].T @ w)
            if np.linalg.norm(w) > tol * nv:
                ok = True
        if not ok:
            f = fill_vector(n, j)
            w = f - Q[:, :j] @ (Q[:, :j].T @ f)
            w = w - Q[:, :j] @ (Q[:, :j].T @ w)
        Q[:, j] = w / np.linalg.norm(w)
    return Q


def qr_pos(Z):
    """Thin QR with diag(R) >= 0 (the unique QR of a full-rank matrix; Eq. ortho-iter)."""
    Q, R = np.linalg.qr(np.asarray(Z, dtype=np.float64))
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :], R * s[:, None]


def orth_iter(op: Operator, Q, iters):
    """Q^(t) R^(t) = P Q^(t-1) (Eq. ortho-iter), ``iters`` times."""
    for _ in range(iters):
        Q, _ = qr_pos(apply_P(op, Q))
    return Q


# --------------------------------------------------------------------------------------
# Discretize (Sec. 7, Definition 2, Eqs. updateY and svd-in-discr, Alg. 5)

def complete_null(B, s, rtol=1e-12):
    """Replace the columns of the orthogonal factor B that belong to (numerically) zero
    singular values by a deterministic completion: for each such column, in order, the
    standard basis vector with the largest residual against the columns before it (the
    smaller index on ties), orthogonalised twice and normalised."""
    B = B.copy()
    k = B.shape[1]
    r = int((s > rtol * s[0]).sum()) if s.shape[0] and s[0] > 0 else 0
    for j in range(r, k):
        E = np.eye(B.shape[0])
        Wr = E - B[:, :j] @ (B[:, :j].T @ E)
        nrm = np.linalg.norm(Wr, axis=0)
        i = int(np.argmax(nrm))
        w = Wr[:, i]
        w = w - B[:, :j] @ (B[:, :j].T @ w)
        B[:, j] = w / np.linalg.norm(w)
    return B


def discretize(Qk, max_iter=30, tol=1e-12, colnorm="l1"):
    """Alternate Y and R (Alg. 5): Y = row-wise argmax of Q~ R (Eq. updateY); Y~ = Y with
    columns divided by their sums; U Omega V^T = SVD(Y~^T Q~); R = V U^T (Eq. svd-in-discr);
    obj = n - 2 trace(Omega); stop when obj no longer changes.

    Readings: Q~ is the row-normalised input (zero rows stay zero); R starts at I_k; argmax
    ties go to the smaller column; column normalisation is the L1 division of Alg. 5 (an
    empty column stays zero); obj "does not change" means |obj - obj_prev| <= tol * max(1,
    |obj|) in FP64; singular vectors of zero singular values are completed by
    complete_null.  Returns (labels, R, obj, iterations)."""
    Q = np.asarray(Qk, dtype=np.float64)
    n, k = Q.shape
    nr = np.sqrt((Q * Q).sum(axis=1))
    Qt = np.zeros_like(Q)
    nz = nr > 0
    Qt[nz] = Q[nz] / nr[nz, None]
    R = np.eye(k)
    obj_prev = None
    obj = None
    labels = None
    it = 0
    for it in range(1, max_iter + 1):
        labels = np.argmax(Qt @ R, axis=1)
        cnt = np.bincount(labels, minlength=k).astype(np.float64)
        Yt = np.zeros((n, k))
        if colnorm == "l1":
            Yt[np.arange(n), labels] = 1.0 / cnt[labels]
        elif colnorm == "l2":
            Yt[np.arange(n), labels] = 1.0 / np.sqrt(cnt[labels])
        else:
            Yt[np.arange(n), labels] = 1.0
        M = Yt.T @ Qt
        U, s, Vt = np.linalg.svd(M)
        U = complete_null(U, s)
        V = complete_null(Vt.T, s)
        R = V @ U.T
        obj = n - 2.0 * s.sum()
        if obj_prev is not None and abs(obj - obj_prev) <= tol * max(1.0, abs(obj)):
            break
        obj_prev = obj
    return labels.astype(np.int64), R, obj, it


# --------------------------------------------------------------------------------------
# Multi-hop conductance (Alg. 2 / Alg. 4, conductance evaluation, Eq. mhc-comp-ancka)

def mhc(op: Operator, labels, k, alpha, gamma):
    """phi = 1 - (1/k) trace(Yh^T F^(gamma)) with F^(0) = alpha Yh and
    F^(l) = (1-alpha) P F^(l-1) + F^(0) (Eq. mhc-comp-ancka).

    Note: with gamma finite the rows of S sum to 1 - (1-alpha)^(gamma+1), so this value
    exceeds Phi of Eq. (mh-cond) by exactly (1-alpha)^(gamma+1); the algorithm's value is
    the one the method compares.

    The trace is summed node by node, sum_i Yh[i, c(i)] F[i, c(i)], so that phi is a function of
    the partition alone: renaming the clusters permutes the columns of F, and each column is
    computed by the same arithmetic, so the summands and their order do not change."""
    labels = np.asarray(labels, dtype=np.int64)
    Yh = normalized_bcm(labels, k)
    F0 = alpha * Yh
    F = F0
    for _ in range(gamma):
        F = (1.0 - alpha) * apply_P(op, F) + F0
    rows = np.arange(labels.shape[0])
    return 1.0 - float(np.sum(Yh[rows, labels] * F[rows, labels])) / k


# --------------------------------------------------------------------------------------
# Whole method (Alg. 4)

@dataclass
class ClusterReport:
    iterations: int = 0
    reason: str = ""
    phi_trace: List[tuple] = field(default_factory=list)   # (t, phi_t)
    best_phi: float = float("inf")
    best_t: int = 0
    init: str = "cold"
    phi_init_cold: float = float("nan")
    phi_init_warm: float = float("nan")


def cluster(op: Operator, k, alpha=0.2, gamma=3, tau=5, T_i=25, T_a=1000, eps_q=0.005,
            disc_max_iter=30, Zwarm=None):
    """Alg. 4 from the initial BCM to the returned labels.

    Readings: Phi(Y^(0)) is evaluated before the loop so that the first comparison
    with the best labels so far has a value; Eq. (tcond-2) is tested on the history [phi_0, phi_tau, phi_2tau, ...]
    once three values exist; the norm of Eq. (tcond-1) is the Frobenius norm of the whole
    block; Discretize gets columns 2..k+1 of Q (the first, constant eigenvector is
    dropped, Sec. 4).  With ``Zwarm`` (n x k), the learned warm start replaces the greedy
    initial BCM when its labels have no larger MHC than the greedy ones."""
    n = op.n
    rep = ClusterReport()
    y_cold, _ = init_bcm(op, k, alpha, T_i)
    phi_cold = mhc(op, y_cold, k, alpha, gamma)
    rep.phi_init_cold = phi_cold
    Y, phi0 = y_cold, phi_cold
    C = np.concatenate([np.full((n, 1), 1.0 / math.sqrt(n)), normalized_bcm(y_cold, k)], axis=1)
    if Zwarm is not None:
        y_warm = np.argmax(np.asarray(Zwarm), axis=1)
        phi_warm = mhc(op, y_warm, k, alpha, gamma)
        rep.phi_init_warm = phi_warm
        if phi_warm <= phi_cold:
            Y, phi0 = y_warm, phi_warm
            rep.init = "warm"
            C = np.concatenate([np.full((n, 1), 1.0 / math.sqrt(n)), np.asarray(Zwarm, dtype=np.float64)], axis=1)
    Q = initial_q(C)
    best, best_phi, best_t = Y, phi0, 0
    hist = [phi0]
    rep.phi_trace.append((0, phi0))
    rep.reason = "max_iter"
    t = 0
    for t in range(1, T_a + 1):
        Qn, _ = qr_pos(apply_P(op, Q))
        dq = float(np.linalg.norm(Qn - Q))
        Q = Qn
        if t % tau == 0:
            yt, _, _, _ = discretize(Q[:, 1:], max_iter=disc_max_iter)
            phi = mhc(op, yt, k, alpha, gamma)
            rep.phi_trace.append((t, phi))
            if phi < best_phi:
                best, best_phi, best_t = yt, phi, t
            hist.append(phi)
            if dq < eps_q:
                rep.reason = "converged"
                break
            if len(hist) >= 3 and hist[-3] < hist[-2] < hist[-1]:
                rep.reason = "early_stop"
                break
    rep.iterations = t
    rep.best_phi = best_phi
    rep.best_t = best_t
    return np.asarray(best, dtype=np.int64), rep
