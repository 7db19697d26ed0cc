"""Workspace lifetime of a handle: buffers replaced after a call was captured into a HIP graph are
kept until cn_destroy (the graph holds their addresses); before any capture they are freed.
Checked from the host through cn_handle_info; the captured graph is never replayed."""
import ctypes

import pytest
import torch

import workloads
from paper_2205_00856_amd import _lib
from paper_2205_00856_amd.api import Layout, _operator

pytestmark = pytest.mark.gpu


def _info(lib, h):
    nbytes, retired, cap = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    assert lib.cn_handle_info(h, ctypes.byref(nbytes), ctypes.byref(retired),
                              ctypes.byref(cap)) == _lib.CN_OK
    return nbytes.value, retired.value, cap.value


def _step(lib, h, L, op, psi, out, stream):
    Lc = L.c()
    return lib.cn_step(h, ctypes.byref(Lc), ctypes.byref(op), 0.0, ctypes.c_void_p(psi.data_ptr()),
                       ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream))


def _case(n, seed):
    w = workloads.random_cn(n, seed)
    dev = torch.device("cuda", 0)
    V = torch.from_numpy(w["V"]).to(dev)
    psi = torch.from_numpy(w["psi"]).to(dev)
    return V, psi, _operator(V, w["dx"], w["dt"]), Layout.contiguous(n, 1)


@pytest.fixture()
def handle():
    lib = _lib.lib()
    h = ctypes.c_void_p()
    assert lib.cn_create(ctypes.byref(h), 0) == _lib.CN_OK
    yield lib, h
    torch.cuda.synchronize()
    assert lib.cn_destroy(h) == _lib.CN_OK


def test_growth_before_capture_frees(handle):
    lib, h = handle
    stream = torch.cuda.current_stream()
    V1, p1, op1, L1 = _case(100_003, 1)
    out1 = torch.empty_like(p1)
    assert _step(lib, h, L1, op1, p1, out1, stream) == _lib.CN_OK
    b1, r1, c1 = _info(lib, h)
    V2, p2, op2, L2 = _case(3_000_017, 2)
    out2 = torch.empty_like(p2)
    assert _step(lib, h, L2, op2, p2, out2, stream) == _lib.CN_OK
    torch.cuda.synchronize()
    b2, r2, c2 = _info(lib, h)
    assert (r1, c1, r2, c2) == (0, 0, 0, 0)
    assert b2 > b1


def test_growth_after_capture_retires(handle):
    lib, h = handle
    V1, p1, op1, L1 = _case(100_003, 3)
    out1 = torch.empty_like(p1)
    Lc = L1.c()
    assert lib.cn_reserve(h, ctypes.byref(Lc)) == _lib.CN_OK
    side = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        assert _step(lib, h, L1, op1, p1, out1, side) == _lib.CN_OK
    _, r0, c0 = _info(lib, h)
    assert (r0, c0) == (0, 1)
    # a larger layout outside capture grows the workspace: the captured graph's buffer is kept
    V2, p2, op2, L2 = _case(3_000_017, 4)
    out2 = torch.empty_like(p2)
    assert _step(lib, h, L2, op2, p2, out2, torch.cuda.current_stream()) == _lib.CN_OK
    torch.cuda.synchronize()
    _, r1, c1 = _info(lib, h)
    assert (r1, c1) == (1, 1)
    del g
