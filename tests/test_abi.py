"""The C-ABI library loads and exports every entry point declared in include/cntri.h (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cntri.h")
LIB = os.path.join(ROOT, "paper_2205_00856_amd", "libcntri.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cn_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("cn_tridiag_solve", "cn_step", "cn_create", "cn_destroy", "cn_reserve",
                     "cn_tridiag_solve_adjoint", "cn_step_adjoint", "cn_propagate",
                     "cn_get_status", "cn_status_string", "cn_assemble", "cn_rhs"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcntri.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcntri.so not built")
def test_python_binding_covers_the_header():
    from paper_2205_00856_amd import _lib

    assert set(_lib.EXPORTED) == set(declared_functions())
    lib = _lib.lib()
    assert lib.cn_status_string(-1).decode() == "CN_ERR_INVALID_ARG"
    assert lib.cn_status_string(1).decode() == "CN_NUMERICAL_BREAKDOWN"
    assert b"gfx950" in lib.cn_version()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcntri.so not built")
def test_null_handle_is_rejected_without_touching_a_gpu():
    from paper_2205_00856_amd import _lib

    lib = _lib.lib()
    L = _lib.CnLayout()
    L.n, L.batch, L.elem_stride, L.batch_stride = 8, 1, 1, 8
    st = lib.cn_tridiag_solve(None, ctypes.byref(L), None, None, None, None, None, None)
    assert st == _lib.CN_ERR_INVALID_ARG
    assert lib.cn_destroy(None) == _lib.CN_ERR_INVALID_ARG
    assert lib.cn_create(None, 0) == _lib.CN_ERR_INVALID_ARG
