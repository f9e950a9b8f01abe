"""Quality measures of the parameter study (CPU): Acc, macro F1, NMI and ARI against planted
labels, pinned on cases with known values."""
import numpy as np

from paper_2408_05459_amd import sweep


def test_quality_of_a_relabelled_partition_is_perfect():
    rng = np.random.default_rng(0)
    truth = rng.integers(0, 5, size=200)
    perm = np.array([3, 0, 4, 1, 2])
    q = sweep.quality(perm[truth], truth, 5)
    assert q == {"acc": 1.0, "f1": 1.0, "nmi": 1.0, "ari": 1.0}


def test_quality_counts_the_best_matching():
    # classes 0, 1 of 4 nodes each; cluster 0 takes 3 of class 0 and 1 of class 1, cluster 1 the rest
    truth = np.array([0, 0, 0, 0, 1, 1, 1, 1])
    pred = np.array([1, 1, 1, 0, 0, 0, 0, 1])
    q = sweep.quality(pred, truth, 2)
    # matching cluster 1 -> class 0 (3 nodes), cluster 0 -> class 1 (3 nodes): Acc 6/8
    assert q["acc"] == 0.75
    # per class: precision 3/4, recall 3/4 -> F1 0.75 for both
    assert abs(q["f1"] - 0.75) < 1e-12


def test_quality_with_an_empty_cluster():
    truth = np.array([0, 0, 1, 1, 2, 2])
    pred = np.array([0, 0, 0, 0, 1, 1])          # cluster 2 empty: class 0 or 1 unmatched
    q = sweep.quality(pred, truth, 3)
    assert abs(q["acc"] - 4 / 6) < 1e-12
    # matched classes: one of {0, 1} with precision 2/4, recall 1 -> 2/3; class 2 -> 1; the third 0
    assert abs(q["f1"] - (2 / 3 + 1.0 + 0.0) / 3) < 1e-12
