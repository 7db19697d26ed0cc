"""cn_tridiag_solve_noalloc (the entry point that allocates no device memory) against
cn_tridiag_solve, through the C ABI: the same layouts must give the same x (same plan, same
kernels), on consecutive calls that share the library's one scratch array, the second call
smaller than the first; a layout larger than the array is refused with nothing enqueued."""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_00856_amd as cn
    from paper_2205_00856_amd import _lib

    cn.handle(0)
    # the breakdown flag is sticky per handle: start from a clear flag, whatever earlier work in
    # this process left on the shared handle, so that the checks below see these calls only
    cn.get_status()
    return torch, cn, _lib


def _system(torch, n, seed, batch=1):
    a, b, c, d = workloads.random_system(n * batch, seed, "herm")
    return tuple(torch.from_numpy(v).cuda() for v in (a, b, c, d))


def _solve(torch, cn, _lib, fn, layout, a, b, c, d):
    x = torch.full_like(d, float("nan"))
    h = cn.handle(0)
    Lc = layout.c()
    st = getattr(_lib.lib(), fn)(h.ptr, ctypes.byref(Lc), ctypes.c_void_p(a.data_ptr()),
                                 ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(c.data_ptr()),
                                 ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.CN_OK, (fn, st)
    return x


def rel(x, y):
    return float(torch_norm(x - y) / torch_norm(y))


def torch_norm(t):
    return float(np.linalg.norm(t.cpu().numpy()))


@pytest.mark.parametrize("sizes", [
    # (n, batch) of two consecutive calls, the second smaller: a multi-level single system
    # then a two-level one; then a batch of whole-tile systems after a long system
    ((3_000_017, 1), (70_001, 1)),
    ((1_000_003, 1), (777, 40)),
])
def test_noalloc_matches_solve_on_consecutive_calls(gpu, oracle_mod, sizes):
    torch, cn, _lib = gpu
    for k, (n, batch) in enumerate(sizes):
        print(f"noalloc call {k}: n={n} batch={batch}", flush=True)
        a, b, c, d = _system(torch, n, 900 + k, batch)
        L = cn.Layout.contiguous(n, batch)
        x_ref = _solve(torch, cn, _lib, "cn_tridiag_solve", L, a, b, c, d)
        x = _solve(torch, cn, _lib, "cn_tridiag_solve_noalloc", L, a, b, c, d)
        torch.cuda.synchronize()
        assert cn.get_status() == 0
        assert bool(torch.isfinite(x).all())
        assert rel(x, x_ref) <= 1e-11
        # the first system against the oracle as well
        ah, bh, ch, dh = (t[:n].cpu().numpy() for t in (a, b, c, d))
        ref = oracle_mod.thomas(ah, bh, ch, dh)
        xh = x[:n].cpu().numpy()
        assert np.linalg.norm(xh - ref) / np.linalg.norm(ref) <= 1e-11


def test_noalloc_in_place_and_python_binding(gpu):
    torch, cn, _lib = gpu
    n = 200_003
    a, b, c, d = _system(torch, n, 950)
    x_ref = cn.solve(a, b, c, d)
    dd = d.clone()
    cn.solve_noalloc(a, b, c, dd, out=dd)  # x aliases d
    torch.cuda.synchronize()
    assert rel(dd, x_ref) <= 1e-11


def test_noalloc_refuses_a_layout_beyond_the_scratch_array(gpu):
    """2^30 rows need more than the fixed array; the refusal happens on the host, before any
    pointer is read, so placeholder (never dereferenced) device pointers are passed."""
    torch, cn, _lib = gpu
    h = cn.handle(0)
    L = cn.Layout.contiguous(1 << 30, 1).c()
    dummy = torch.zeros(1, dtype=torch.complex128, device="cuda")
    p = ctypes.c_void_p(dummy.data_ptr())
    st = _lib.lib().cn_tridiag_solve_noalloc(h.ptr, ctypes.byref(L), p, p, p, p, p,
                                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.CN_ERR_SCRATCH_TOO_SMALL
    assert _lib.lib().cn_status_string(st).decode() == "CN_ERR_SCRATCH_TOO_SMALL"
    torch.cuda.synchronize()
    assert cn.get_status() == 0
