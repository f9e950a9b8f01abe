"""GPU: the two-pass BF16 KNN scan (window pass + symmetric pass + hand-over merge).

The result of the scan may not depend on how the pairs are split between the passes: the
final lists for windows of +-1, +-4 and +-9 blocks, for the default windows (the blocks of each
row's coarse cell), for the whole-ring scan (no symmetric pass) and after a forced overflow of
the hand-over buffer (which redoes the scan whole) must be identical, and sampled rows must match
the oracle's exact search.  Block counts odd and even
(the opposite block of an even ring is scanned from one side only), a ragged last block and
zero rows are covered.
"""
import numpy as np
import pytest

from paper_2408_05459_amd import synth
from tests.helpers import check_knn_rows, gamma_d

pytestmark = pytest.mark.gpu

QB = 256   # rows per block (workgroup) of the d = 128 scan


def data(n, seed, zero_rows=()):
    rng = np.random.default_rng(seed)
    labels = synth.planted_labels(n, 12, rng)
    X = synth.gmm_attributes(labels, synth.gmm_centres(12, 128, 1.5, rng), rng, "bf16")
    X[list(zero_rows)] = 0
    return X


def run(lib, X, K, monkeypatch, window=None, handover=None):
    import torch
    from paper_2408_05459_amd.binding import upload_attributes
    monkeypatch.delenv("ANCKA_KNN_WINDOW", raising=False)
    monkeypatch.delenv("ANCKA_KNN_HANDOVER", raising=False)
    if window is not None:
        monkeypatch.setenv("ANCKA_KNN_WINDOW", str(window))
    if handover is not None:
        monkeypatch.setenv("ANCKA_KNN_HANDOVER", str(handover))
    idx, sim, st = lib.knn(upload_attributes(X, "bf16"), K, "bf16")
    torch.cuda.synchronize()
    return idx.cpu().numpy(), sim.cpu().numpy(), st


def sym_pairs(nwg, w):
    """Unordered row pairs of the symmetric pass with windows of +-w blocks."""
    blocks = 0
    for i in range(nwg):
        hb = nwg // 2 - 1 if (nwg % 2 == 0 and i >= nwg // 2) else nwg // 2
        blocks += max(0, hb - w)
    return blocks * QB * QB


@pytest.mark.parametrize("n", [20000, 20380])          # 79 blocks (odd), 80 blocks (even, ragged)
def test_split_of_pairs_does_not_change_lists(lib, monkeypatch, n):
    K = 10
    zero = [7, 5000, n - 1]
    X = data(n, 11 + n % 7, zero)
    nwg = -(-n // QB)
    gi_full, gs_full, st_full = run(lib, X, K, monkeypatch, window=nwg)
    assert st_full.window == -1 and st_full.sym_ms == 0.0
    for w in (1, 4, 9, None):
        gi, gs, st = run(lib, X, K, monkeypatch, window=w)
        print(f"n={n} w={w}: window {st.window} handed over {st.handed_over}, sym {st.sym_ms:.2f} ms, "
              f"uncertified {st.uncertified_rows}")
        assert st.rescanned == 0 and st.handed_over > 0 and st.window > 0
        if w is not None:
            assert st.window == 2 * w + 1
            assert st.sym_pairs == sym_pairs(nwg, w)
        assert np.array_equal(gi, gi_full), f"w={w}: lists differ from the whole-ring scan"
        assert np.array_equal(gs, gs_full)
    assert st_full.zero_rows == len(zero)
    for z in zero:
        assert np.all(gi_full[z] == -1)
    rows = np.sort(np.random.default_rng(n).choice(np.setdiff1d(np.arange(n), zero), 300, replace=False))
    swaps = check_knn_rows(X.astype(np.float32), rows, gi_full[rows], gs_full[rows], K, 2 * gamma_d(128, 2.0 ** -24))
    assert swaps <= 1


def test_handover_overflow_rescans(lib, monkeypatch):
    n, K = 9000, 8
    X = data(n, 5)
    gi_a, gs_a, st_a = run(lib, X, K, monkeypatch, window=2)
    assert st_a.rescanned == 0 and st_a.handed_over > 1
    gi_b, gs_b, st_b = run(lib, X, K, monkeypatch, window=2, handover=1)
    assert st_b.rescanned == 1 and st_b.window == -1
    assert np.array_equal(gi_a, gi_b) and np.array_equal(gs_a, gs_b)


def test_default_window_uses_symmetric_pass(lib, monkeypatch):
    n = 40000
    X = data(n, 9)
    gi, gs, st = run(lib, X, 10, monkeypatch)
    nwg = -(-n // QB)
    assert 0 < st.window <= nwg // 4 and st.rescanned == 0
    assert 0 < st.sym_pairs <= sym_pairs(nwg, 0)
    rows = np.sort(np.random.default_rng(1).choice(n, 200, replace=False))
    assert check_knn_rows(X.astype(np.float32), rows, gi[rows], gs[rows], 10, 2 * gamma_d(128, 2.0 ** -24)) <= 1


@pytest.mark.parametrize("K", [10, 11, 16, 20, 21])
def test_list_lengths_around_the_bound_pass(lib, monkeypatch, K):
    # the window pass starts from the bound pass's lower bounds: 11 values per lane bound lists up
    # to 2K = 21, 21 values lists up to 41; longer lists (K = 21) skip the bound pass
    n = 9000
    X = data(n, 21 + K)
    gi_w, gs_w, st_w = run(lib, X, K, monkeypatch, window=2)
    gi_f, gs_f, st_f = run(lib, X, K, monkeypatch, window=n)
    assert st_w.window == 5 and st_f.window == -1
    assert np.array_equal(gi_w, gi_f) and np.array_equal(gs_w, gs_f)
    rows = np.sort(np.random.default_rng(K).choice(n, 150, replace=False))
    assert check_knn_rows(X.astype(np.float32), rows, gi_f[rows], gs_f[rows], K, 2 * gamma_d(128, 2.0 ** -24)) <= 1
