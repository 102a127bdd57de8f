"""The C-ABI library loads on the CPU and exports every function declared in
include/mtgp.h (no compute calls: there is no GPU here)."""
import ctypes
import os

import pytest

from paper_2603_16014_amd import _lib


def test_header_declares_the_boundary():
    names = _lib.header_functions()
    for required in ("mtgp_gen_points", "mtgp_kernel_cols", "mtgp_fwht", "mtgp_fft", "mtgp_nll",
                     "mtgp_nll_grad", "mtgp_predict", "mtgp_set_data", "mtgp_plan_create"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _lib.header_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the Python binding declares exactly the header's functions
    assert sorted(_lib.SIGNATURES) == _lib.header_functions()


@pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="library not built")
def test_strerror_without_device():
    lib = _lib.load()
    assert lib.mtgp_strerror(0) == b"ok"
    assert b"positive definite" in lib.mtgp_strerror(-2)
