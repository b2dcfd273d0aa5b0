"""CPU checks of the C ABI: the built library loads and exports every function the header declares.

No compute call is made (there is no GPU on this host).
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastlsq.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(flsq_[a-z_A-Z0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("flsq_solve_linear", "flsq_factorize", "flsq_factor_solve", "flsq_evaluate", "flsq_solve_newton",
                 "flsq_gram", "flsq_inverse_loss_grad"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2602_10541_amd import fastlsq
    if not os.path.exists(fastlsq.LIB_PATH):
        pytest.skip("library not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(fastlsq.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_declared()) == set(fastlsq.EXPORTS)
    assert b"gfx950" in fastlsq.load().flsq_build_info()


def test_binding_structs_match_header_layout():
    """ctypes mirrors of the ABI structs have the C sizes implied by the header's field lists."""
    from paper_2602_10541_amd import fastlsq as fl
    assert ctypes.sizeof(fl.flsq_term) == 16
    assert ctypes.sizeof(fl.flsq_op) == 16
    assert ctypes.sizeof(fl.flsq_basis) == 32
    assert ctypes.sizeof(fl.flsq_rows) == 48
    assert ctypes.sizeof(fl.flsq_solve_opts) == 32
    assert ctypes.sizeof(fl.flsq_solve_info) == 8 + 8 * 9
    assert ctypes.sizeof(fl.flsq_newton_opts) == 32 + 8 + 8 + 8 + 8


def test_no_gpu_means_loud_failure():
    """Without a GPU the binding raises; it never falls back to the CPU."""
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_2602_10541_amd import fastlsq
    if not os.path.exists(fastlsq.LIB_PATH):
        pytest.skip("library not built")
    with pytest.raises(RuntimeError):
        fastlsq.Context(0)
