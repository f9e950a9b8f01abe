"""CPU checks of the C-ABI boundary: the library loads and exports every declared entry point
(no compute call without a GPU), and the binding declares the same set."""
import ctypes
import os

import pytest

from tests.helpers import declared_symbols

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ancka.h")
LIB = os.path.join(ROOT, "paper_2408_05459_amd", "libancka.so")


def test_header_declares_the_boundary():
    names = declared_symbols(HEADER)
    for required in ["ancka_knn", "ancka_build_operator", "ancka_orth_iter", "ancka_discretize", "ancka_cluster",
                     "ancka_mhc", "ancka_init_bcm", "ancka_create", "ancka_destroy"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_symbols(HEADER):
        assert hasattr(lib, name), name


def test_binding_matches_header():
    from paper_2408_05459_amd import binding
    assert binding.EXPORTED == declared_symbols(HEADER)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_default_params_are_the_papers():
    from paper_2408_05459_amd import binding
    lib = binding.Lib(LIB)
    p = lib.ancka_default_params()
    assert (p.K, p.alpha, p.beta, p.gamma, p.tau, p.T_i, p.T_a, p.eps_q) == (10, 0.2, 0.5, 3, 5, 25, 1000, 0.005)
    assert p.k == 0 and p.early_stop == 1


def test_missing_library_fails_loudly(tmp_path):
    from paper_2408_05459_amd import binding
    with pytest.raises(RuntimeError, match="not found"):
        binding.Lib(str(tmp_path / "libancka.so"))
