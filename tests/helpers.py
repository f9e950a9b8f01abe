"""Shared test utilities: oracle-side reference builds and tolerance-aware comparisons."""
from __future__ import annotations

import math
import re

import numpy as np

import oracle


def gamma_d(d: int, u: float) -> float:
    """Higham's dot-product rounding bound gamma_d = d u / (1 - d u)."""
    return d * u / (1.0 - d * u)


def check_knn_rows(X, rows, gpu_idx, gpu_sim, K, tol):
    """Tie-aware KNN parity on the given rows.

    With the oracle's FP64 similarities s_i. and its K-th value s_K, the GPU set G_i is accepted
    iff {j : s_ij > s_K + tol} is a subset of G_i, which is a subset of {j : s_ij >= s_K - tol};
    every returned similarity must match the oracle's within tol, and the list must be ordered.
    Returns the number of rows whose set differs from the oracle's by a tie swap."""
    S = oracle.cosine_rows(X, rows)
    ref_i, ref_s = oracle.knn(X, K, rows=rows)
    swaps = 0
    for t, i in enumerate(rows):
        g = [int(j) for j in gpu_idx[t] if j >= 0]
        gs = [float(v) for j, v in zip(gpu_idx[t], gpu_sim[t]) if j >= 0]
        r = [int(j) for j in ref_i[t] if j >= 0]
        assert len(g) == len(r), f"row {i}: {len(g)} neighbours, oracle {len(r)}"
        assert len(set(g)) == len(g), f"row {i}: duplicate neighbours"
        if not r:
            continue
        assert i not in g
        sK = S[t][r[-1]]
        must = set(np.nonzero(S[t] > sK + tol)[0].tolist())
        may = set(np.nonzero(S[t] >= sK - tol)[0].tolist())
        assert must <= set(g) <= may, f"row {i}: set outside tie tolerance"
        for j, v in zip(g, gs):
            assert abs(v - S[t][j]) <= tol + 1e-7 * abs(S[t][j]), f"row {i}: sim of {j} {v} vs {S[t][j]}"
        assert all(gs[a] >= gs[a + 1] - tol for a in range(len(gs) - 1)), f"row {i}: not ordered"
        if set(g) != set(r):
            swaps += 1
    return swaps


def principal_sin(A, B):
    """sin of the largest principal angle between span(A) and span(B) (Bjorck & Golub 1973)."""
    Qa, _ = np.linalg.qr(np.asarray(A, dtype=np.float64))
    Qb, _ = np.linalg.qr(np.asarray(B, dtype=np.float64))
    return float(np.linalg.norm(Qb - Qa @ (Qa.T @ Qb), 2))


def oracle_operator(net, K, beta, knn=None):
    """Oracle KNN (unless given) and operator for a synth.Network."""
    _, zero = oracle.normalize_rows(net.X)
    if knn is None:
        knn = oracle.knn(net.X, K)
    ki, ks = knn
    op = oracle.build_operator(net.kind, net.n, net.ptrs, net.idxs, net.m, zero, ki, ks, beta)
    return op, ki, ks


def ari(a, b) -> float:
    from sklearn.metrics import adjusted_rand_score
    return float(adjusted_rand_score(np.asarray(a), np.asarray(b)))


def declared_symbols(header_path: str):
    """Function names declared in the C header."""
    txt = open(header_path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:[a-z_]+\s*\*?\s+)+\**(ancka_[a-z0-9_]+)\s*\(", txt, flags=re.M)))
