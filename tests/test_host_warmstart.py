"""Host-side logic of the warm-start driver (CPU): the cluster-to-centre assignment of the
product code against the oracle's, on seeded mixtures."""
import numpy as np
import pytest

import oracle
from paper_2408_05459_amd import synth, warmstart


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_centre_assignment_matches_oracle(seed):
    net, _ = synth.make_warm_graph(1500, 5200 + seed, k=30, d=512)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(30)
    labels = perm[net.labels]               # clusters numbered in a scrambled order
    centres = synth.warm_centres()
    got = warmstart.centre_assignment(net.X, labels, centres)
    Xh, _ = oracle.normalize_rows(net.X)
    want = oracle.centre_map(labels, Xh, centres)
    assert np.array_equal(got, want)
    # cluster perm[c] holds the nodes generated from centre c
    assert np.array_equal(got[perm], np.arange(30))


def test_centre_assignment_with_empty_cluster():
    net, _ = synth.make_warm_graph(600, 5300, k=30, d=512)
    labels = net.labels.copy()
    labels[labels == 7] = 8                 # cluster 7 empty
    centres = synth.warm_centres()
    got = warmstart.centre_assignment(net.X, labels, centres)
    Xh, _ = oracle.normalize_rows(net.X)
    assert sorted(got) == list(range(30))
    assert np.array_equal(got, oracle.centre_map(labels, Xh, centres))
