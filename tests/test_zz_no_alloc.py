"""ancka_discretize_noalloc (state in the library's static device array) against
ancka_discretize (context workspace), through the C ABI: same kernels, so labels, R, the
objective and the step count must be bitwise equal, on two calls in a row with the second
input smaller, and on calls interleaved with the allocating entry point."""
import numpy as np
import pytest
import scipy.linalg

pytestmark = pytest.mark.gpu


def planted(n, k, noise, seed):
    rng = np.random.default_rng(seed)
    y = rng.integers(0, k, size=n)
    A = rng.standard_normal((k, k)) * 0.15
    R0 = np.eye(k)[rng.permutation(k)] @ scipy.linalg.expm(A - A.T)
    return np.eye(k)[y] @ R0 + noise * rng.standard_normal((n, k))


def block(Qh, ld, dtype):
    import torch
    full = np.zeros((Qh.shape[0], ld))
    full[:, 1:Qh.shape[1] + 1] = Qh
    return torch.from_numpy(full).to(torch.float64 if dtype == "f64" else torch.float32).cuda()


def same(a, b):
    (la, Ra, oa, ia), (lb, Rb, ob, ib) = a, b
    assert np.array_equal(la.cpu().numpy(), lb.cpu().numpy())
    assert np.array_equal(Ra, Rb)
    assert oa == ob and ia == ib


CASES = [  # (n, k, ld, dtype, noise, seed): the second input of each pair is smaller
    (200_000, 50, 64, "f32", 0.2, 1),
    (3_000, 7, 8, "f64", 0.05, 2),
]


def test_noalloc_two_calls_in_a_row_match_discretize(lib):
    inputs = [block(planted(n, k, z, s), ld, dt) for n, k, ld, dt, z, s in CASES]
    got = [lib.discretize(T[:, 1:], k, noalloc=True) for T, (_, k, *_) in zip(inputs, CASES)]
    ref = [lib.discretize(T[:, 1:], k) for T, (_, k, *_) in zip(inputs, CASES)]
    for g, r, (n, k, *_) in zip(got, ref, CASES):
        same(g, r)
        assert g[0].shape[0] == n and int(g[0].max()) < k and g[3] >= 2


def test_noalloc_interleaved_with_allocating_calls(lib):
    T1 = block(planted(50_000, 30, 0.3, 3), 32, "f32")
    T2 = block(planted(5_000, 12, 0.1, 4), 16, "f32")
    a = lib.discretize(T1[:, 1:], 30, noalloc=True)
    b = lib.discretize(T2[:, 1:], 12)
    c = lib.discretize(T2[:, 1:], 12, noalloc=True)
    d = lib.discretize(T1[:, 1:], 30)
    same(a, d)
    same(b, c)


def test_noalloc_rejects_k_beyond_its_state(lib):
    from paper_2408_05459_amd.binding import AnckaError
    T = block(np.ones((100, 65)), 68, "f32")
    with pytest.raises(AnckaError, match="ancka_discretize_noalloc"):
        lib.discretize(T[:, 1:], 65, noalloc=True)
