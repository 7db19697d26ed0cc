"""GPU parity of batches that share one matrix (cn_layout.shared_coefficients = 1): several
right-hand sides of one tridiagonal system, and several states under one potential, against the
CPU oracle per right-hand side.  The coefficients of the other systems' positions are filled
with NaN where the layout has room for them, so any read of them would show.

Tolerance: relative L2 <= 1e-11 (FP64 on both sides; rounding only).
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
TOL = 1e-11


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_00856_amd as cn

    cn.handle(0)
    return torch, cn


def rel(x, y):
    x = np.asarray(x)
    y = np.asarray(y)
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))


def to_dev(torch, *arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def log(*a):
    print(*a, flush=True)


# (1 << 20, 5): 1024 tiles, so every workgroup takes all 5 right-hand sides (an odd count of
# them, through both prefetch buffers); (1_000_003, 3): workgroups of 2, the second one short
@pytest.mark.parametrize("n,nrhs", [(1, 3), (1000, 7), (4096, 5), (70_001, 6), (300_007, 16),
                                    (1_000_003, 3), (5000, 33), (1 << 20, 5)])
def test_solve_one_matrix_many_rhs_contiguous(gpu, oracle_mod, n, nrhs):
    torch, cn = gpu
    log("shared solve", n, nrhs)
    a, b, c, _ = workloads.random_system(n, 40 + n, "dd")
    g = np.random.default_rng(n)
    d = workloads.complex_normal(g, nrhs * n)
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    L = cn.Layout.contiguous(n, nrhs, shared_coefficients=True)
    assert "rhs/wg=" in cn.describe_plan(L)  # the matrix is loaded once per tile
    if n == 1 << 20:
        assert f"rhs/wg={nrhs}" in cn.describe_plan(L)
    xt = cn.solve(ta, tb, tc, td, layout=L)
    x = xt.cpu().numpy()
    for s in range(nrhs):
        ref = oracle_mod.thomas(a, b, c, d[s * n:(s + 1) * n])
        assert rel(x[s * n:(s + 1) * n], ref) <= TOL
    # the same rows through the per-system kernels (matrix copied per right-hand side): the
    # same arithmetic, so the same bits
    A, B, C = (t.repeat(nrhs) for t in (ta, tb, tc))
    xr = cn.solve(A, B, C, td, layout=cn.Layout.contiguous(n, nrhs))
    assert torch.equal(xt, xr)
    assert cn.get_status() == 0


@pytest.mark.parametrize("partition,rpt", [(256, 2), (512, 2), (2048, 8)])
def test_solve_one_matrix_many_rhs_tile_shapes(gpu, oracle_mod, partition, rpt):
    """The factored tile at other lane-block sizes (2 rows per lane over 2 and 4 wavefronts, 8
    rows over 4): parity with the oracle and the same bits as the per-system kernels."""
    torch, cn = gpu
    n, nrhs = 100_003, 5
    log("shared solve, tile shape", partition, rpt)
    a, b, c, _ = workloads.random_system(n, 77, "dd")
    g = np.random.default_rng(partition + rpt)
    d = workloads.complex_normal(g, nrhs * n)
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    kw = dict(partition=partition, rows_per_thread=rpt)
    L = cn.Layout.contiguous(n, nrhs, shared_coefficients=True, **kw)
    assert "rhs/wg=" in cn.describe_plan(L)
    xt = cn.solve(ta, tb, tc, td, layout=L)
    x = xt.cpu().numpy()
    for s in (0, nrhs - 1):
        assert rel(x[s * n:(s + 1) * n], oracle_mod.thomas(a, b, c, d[s * n:(s + 1) * n])) <= TOL
    A, B, C = (t.repeat(nrhs) for t in (ta, tb, tc))
    xr = cn.solve(A, B, C, td, layout=cn.Layout.contiguous(n, nrhs, **kw))
    assert torch.equal(xt, xr)
    assert cn.get_status() == 0


def test_solve_one_matrix_many_rhs_interleaved(gpu, oracle_mod):
    """Interleaved right-hand sides (elem_stride = batch): the coefficients are read at system
    0's elements 0, batch, 2 batch, ...; every other element of a, b, c holds NaN."""
    torch, cn = gpu
    n, nrhs = 3000, 70
    a1, b1, c1, _ = workloads.random_system(n, 77, "herm")
    A = np.full((n, nrhs), np.nan + 1j * np.nan)
    B, C = A.copy(), A.copy()
    A[:, 0], B[:, 0], C[:, 0] = a1, b1, c1
    g = np.random.default_rng(78)
    D = workloads.complex_normal(g, n * nrhs).reshape(n, nrhs)
    ta, tb, tc, td = to_dev(torch, A.ravel(), B.ravel(), C.ravel(), D.ravel())
    L = cn.Layout.interleaved(n, nrhs, shared_coefficients=True)
    log("interleaved shared plan:", cn.describe_plan(L))
    x = cn.solve(ta, tb, tc, td, layout=L).cpu().numpy().reshape(n, nrhs)
    for s in range(nrhs):
        assert rel(x[:, s], oracle_mod.thomas(a1, b1, c1, D[:, s])) <= TOL
    assert cn.get_status() == 0


@pytest.mark.parametrize("n", [2048, 100_003])
def test_step_and_propagate_one_potential(gpu, oracle_mod, n):
    """Several states under one potential and field: one step, then a fused propagation."""
    torch, cn = gpu
    nst, dx, dt, steps = 4, 0.05, 0.01, 3
    g = np.random.default_rng(n + 5)
    V = g.uniform(-2.0, 0.0, n)
    xg = workloads.grid_1d(n, dx)
    E = g.normal(0.0, 0.05, steps)
    psi = workloads.complex_normal(g, nst * n)
    tV, txg, tpsi = to_dev(torch, V, xg, psi)
    L = cn.Layout.contiguous(n, nst, shared_coefficients=True)
    out = cn.step(tpsi, tV, dx, dt, E=E[0], xgrid=txg, layout=L).cpu().numpy()
    for s in range(nst):
        ref = oracle_mod.cn_step(psi[s * n:(s + 1) * n], V, dx, dt, xg, E[0])
        assert rel(out[s * n:(s + 1) * n], ref) <= TOL
    cn.propagate(tpsi, tV, dx, dt, steps, E=E, xgrid=txg, layout=L)
    res = tpsi.cpu().numpy()
    for s in range(nst):
        ref = oracle_mod.cn_propagate(psi[s * n:(s + 1) * n], V, dx, dt, steps, xg, E)
        assert rel(res[s * n:(s + 1) * n], ref) <= TOL


def test_shared_coefficients_refused_where_undefined(gpu):
    """Entry points that accumulate per-system gradients or materialise per-system arrays
    return CN_ERR_UNSUPPORTED for a shared layout and launch nothing."""
    torch, cn = gpu
    from paper_2205_00856_amd import _lib

    n, nst = 500, 3
    g = np.random.default_rng(9)
    psi = to_dev(torch, workloads.complex_normal(g, nst * n))[0]
    V = to_dev(torch, g.uniform(-1, 0, nst * n))[0]
    L = cn.Layout.contiguous(n, nst, shared_coefficients=True)
    calls = [
        lambda: cn.rhs(psi, V, 0.1, 0.01, layout=L),
        lambda: cn.assemble(V, 0.1, 0.01, layout=L),
        lambda: cn.solve_adjoint(psi, psi, psi, psi, psi, layout=L),
        lambda: cn.step_adjoint(psi, psi, psi, V, 0.1, 0.01, layout=L),
    ]
    for call in calls:
        with pytest.raises(_lib.CnError, match="UNSUPPORTED"):
            call()
    torch.cuda.synchronize()
    assert cn.get_status() == 0
