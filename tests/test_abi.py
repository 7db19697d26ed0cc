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


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcntri.so not built")
def test_layout_errors_are_reported_on_the_host():
    """Error paths of the boundary, forced from the host (no GPU needed)."""
    import numpy as np

    from paper_2205_00856_amd import _lib

    lib = _lib.lib()
    BAD, UNSUP, OK = _lib.CN_ERR_INVALID_ARG, _lib.CN_ERR_UNSUPPORTED, _lib.CN_OK

    def L(n=10, batch=1, es=1, bs=10, offsets=None, partition=0, rpt=0, shared=0, levels=0):
        x = _lib.CnLayout()
        x.n, x.batch, x.elem_stride, x.batch_stride = n, batch, es, bs
        x.partition, x.rows_per_thread = partition, rpt
        x.shared_coefficients = shared
        x.levels = levels
        if offsets is not None:
            o = np.ascontiguousarray(offsets, dtype=np.int64)
            x.offsets = o.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            x._keep = o
        return x

    def check(layout):
        return lib.cn_check_layout(ctypes.byref(layout))

    assert lib.cn_check_layout(None) == BAD
    assert check(L()) == OK
    assert check(L(n=0)) == BAD
    assert check(L(batch=0)) == BAD
    assert check(L(es=0)) == BAD
    assert check(L(n=10, batch=3, es=1, bs=5)) == BAD      # systems overlap
    assert check(L(n=10, batch=3, es=3, bs=1)) == OK       # interleaved
    assert check(L(n=10, batch=3, es=2, bs=1)) == BAD      # interleaved but overlapping
    assert check(L(n=10, batch=3, es=1, bs=10)) == OK
    assert check(L(offsets=[0, 5, 5, 9], batch=3)) == OK
    assert check(L(offsets=[1, 5, 9], batch=2)) == BAD     # must start at 0
    assert check(L(offsets=[0, 5, 4], batch=2)) == BAD     # decreasing
    assert check(L(offsets=[0, 0], batch=1)) == BAD        # no rows at all
    assert check(L(partition=100)) == BAD                  # not a power of two
    assert check(L(partition=16)) == BAD
    assert check(L(partition=1024, rpt=3)) == BAD
    assert check(L(partition=1024, rpt=16)) == OK
    assert check(L(levels=3)) == OK
    assert check(L(levels=8)) == OK
    assert check(L(levels=9)) == BAD
    assert check(L(levels=-1)) == BAD
    assert check(L(n=1 << 41)) == UNSUP
    assert check(L(n=10, batch=3, es=1, bs=10, shared=1)) == OK   # one matrix, 3 right-hand sides
    assert check(L(shared=2)) == BAD
    assert check(L(offsets=[0, 5, 9], batch=2, shared=1)) == UNSUP


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of cn_layout and cn_operator have the C structs' size and field
    offsets (the header compiled by the host C compiler)."""
    import shutil
    import subprocess

    from paper_2205_00856_amd._lib import CnLayout, CnOperator

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"cn_layout": CnLayout, "cn_operator": CnOperator}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "cntri.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    for line in out.splitlines():
        cname, field, value = line.split()
        py = structs[cname]
        want = ctypes.sizeof(py) if field == "size" else getattr(py, field).offset
        assert int(value) == want, (cname, field)
