"""Pins of the oracle's attribute prologue, KNN and A_K (CPU only)."""
import json
import math
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def brute_knn(X, K, digits=None):
    """Sec. 3.1 written out with Python floats: cosine, self excluded, key (-f, j).
    With ``digits`` the similarity is rounded first, so values equal up to rounding noise
    tie and fall back to the index order."""
    n = len(X)
    norms = [math.sqrt(sum(v * v for v in row)) for row in X]
    out = []
    for i in range(n):
        if norms[i] == 0:
            out.append([-1] * K)
            continue
        cand = []
        for j in range(n):
            if j == i or norms[j] == 0:
                continue
            dot = sum(a * b for a, b in zip(X[i], X[j]))
            sq_i = sum(v * v for v in X[i])
            sq_j = sum(v * v for v in X[j])
            f = dot / math.sqrt(sq_i * sq_j)
            cand.append((-(round(f, digits) if digits else f), j))
        cand.sort()
        out.append([j for _, j in cand[:K]] + [-1] * max(0, K - len(cand)))
    return out


def test_figure1_example():
    fx = json.load(open(os.path.join(HERE, "golden", "figure1.json")))
    X = np.array(fx["attributes"], dtype=np.float64)
    names = fx["nodes"]
    K = fx["from_paper"]["K"]
    idx, sim = oracle.knn(X, K)
    v2 = names.index("v2")
    got = {names[j] for j in idx[v2]}
    assert got == set(fx["from_paper"]["knn_of_v2"])
    S = oracle.cosine_rows(X, [v2])[0]
    for name, val in fx["from_paper"]["cosine_to_v2"].items():
        assert abs(S[names.index(name)] - val) < 1e-12
    # v7 is excluded although its similarity is positive (the distortion example)
    assert names.index("v7") not in idx[v2]
    assert S[v2] == -np.inf


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_knn_matches_brute_force_gaussian(seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((40, 6))
    X[5] = 0.0                       # zero attribute row
    X[7] = X[3] * 2.5                # duplicate direction: cosine 1, still a valid neighbour
    K = 4
    idx, sim = oracle.knn(X, K)
    ref = brute_knn(X.tolist(), K, digits=12)
    for i in range(40):
        if i == 5:
            assert (idx[i] == -1).all() and (sim[i] == 0).all()
            continue
        # 3 and 7 tie up to rounding: compare by rounded key, index order within ties
        got = sorted(zip(np.round(-sim[i], 12).tolist(), idx[i].tolist()))
        assert [j for _, j in got] == ref[i]
        assert 5 not in idx[i] and i not in idx[i]
    assert 7 in idx[3] and abs(sim[3][list(idx[3]).index(7)] - 1.0) < 1e-12


def test_knn_ties_broken_by_index_binary():
    rng = np.random.default_rng(3)
    X = (rng.random((30, 8)) < 0.3).astype(np.float64)
    X[10] = X[4]
    X[20] = X[4]
    X[0] = 0.0
    K = 5
    idx, _ = oracle.knn(X, K)
    ref = brute_knn(X.tolist(), K)
    for i in range(30):
        if i == 0:
            continue
        assert idx[i].tolist() == ref[i]


def test_knn_fewer_candidates_than_K():
    X = np.array([[1.0, 0], [0, 1.0], [1.0, 1.0], [0, 0]])
    idx, sim = oracle.knn(X, 5)
    assert idx[0].tolist()[:2] == [2, 1] and idx[0].tolist()[2:] == [-1, -1, -1]
    assert (idx[3] == -1).all()


def test_knn_rows_subset_equals_full():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((300, 12))
    full_i, full_s = oracle.knn(X, 7)
    rows = np.array([0, 17, 299, 150])
    sub_i, sub_s = oracle.knn(X, 7, rows=rows, block=3)
    assert (sub_i == full_i[rows]).all()
    assert np.allclose(sub_s, full_s[rows], rtol=1e-14, atol=0)


def test_normalize_rows():
    X = np.array([[3.0, 4.0], [0.0, 0.0], [-1.0, 0.0]])
    Xh, zero = oracle.normalize_rows(X)
    assert np.allclose(Xh, [[0.6, 0.8], [0, 0], [-1, 0]], atol=0, rtol=1e-15)
    assert zero.tolist() == [False, True, False]


def test_knn_adjacency_eq_AK_cases():
    # node 0 <-> 1 mutual (2f), 2 -> 1 one-way (f), 3 -> 2 negative (dropped), -1 padding
    nbr_idx = np.array([[1, -1], [0, -1], [1, -1], [2, -1]])
    nbr_sim = np.array([[0.5, 0], [0.5, 0], [0.3, 0], [-0.1, 0]])
    A = oracle.knn_adjacency(4, nbr_idx, nbr_sim).toarray()
    expect = np.zeros((4, 4))
    expect[0, 1] = expect[1, 0] = 1.0
    expect[1, 2] = expect[2, 1] = 0.3
    assert np.array_equal(A, expect)


def test_knn_adjacency_symmetric_nonnegative():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((200, 5))
    idx, sim = oracle.knn(X, 6)
    A = oracle.knn_adjacency(200, idx, sim)
    D = A - A.T
    assert abs(D).max() == 0.0
    assert A.data.min() > 0
    # mutual pairs carry 2f, one-way pairs f
    for i in range(0, 200, 17):
        for t in range(6):
            j = idx[i, t]
            if sim[i, t] <= 0:
                continue
            mutual = i in idx[j]
            assert math.isclose(A[i, j], (2 if mutual else 1) * sim[i, t], rel_tol=1e-15)


@pytest.mark.parametrize("width", [3, 16, 41])
def test_knn_sliced_threshold_matches_brute_force(width):
    """The lower bound t0 taken from the first ``width`` columns never drops a member of the
    top K: narrow slices (one narrower than K, so t0 = -inf) give the brute-force lists,
    including exact ties of duplicated binary rows."""
    rng = np.random.default_rng(6)
    X = (rng.random((90, 10)) < 0.35).astype(np.float64)
    X[30] = X[2]
    X[61] = X[2]
    X[7] = 0.0
    K = 5
    idx, sim = oracle.knn(X, K, width=width, block=17)
    ref = brute_knn(X.tolist(), K)
    for i in range(90):
        if i == 7:
            assert (idx[i] == -1).all()
            continue
        assert idx[i].tolist() == ref[i], i
    full_i, full_s = oracle.knn(X, K)
    assert np.array_equal(idx, full_i) and np.array_equal(sim, full_s)
