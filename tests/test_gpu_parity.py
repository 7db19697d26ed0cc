"""GPU parity: the HIP N-shaped path against the CPU oracle, through the C ABI.

Tolerance: relative L2 <= 1e-11 on complex128 (the workloads' stated bar).  Both sides are
FP64; differences are rounding only (the method reaches x = T^{-1} d exactly, Appendix I).
Sizes span several tiles, ragged tails, nested interface levels and the degenerate cases
(n = 1, one row past a tile, a tile holding the whole system).
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


# ------------------------------------------------------------------ cn_tridiag_solve
@pytest.mark.parametrize("n", [1, 2, 3, 5, 64, 65, 127, 128, 129, 255, 256, 257, 1000, 1024,
                               1025, 4095, 4096, 4097, 10_000, 65_537, 1_000_003, 3_000_017])
@pytest.mark.parametrize("kind", ["dd", "herm"])
def test_solve_single_system(gpu, oracle_mod, n, kind):
    torch, cn = gpu
    log("solve", n, kind)
    a, b, c, d = workloads.random_system(n, 1000 + n, kind)
    ref = oracle_mod.thomas(a, b, c, d)
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    x = cn.solve(ta, tb, tc, td)
    torch.cuda.synchronize()
    assert rel(x.cpu().numpy(), ref) <= TOL
    assert cn.get_status() == 0


@pytest.mark.parametrize("T,M", [(64, 0), (128, 2), (256, 4), (512, 4), (512, 8), (1024, 4),
                                 (1024, 8), (2048, 4), (2048, 8), (4096, 8), (8192, 0),
                                 (16384, 0)])
def test_solve_partition_sweep(gpu, oracle_mod, T, M):
    """Every first-level partition of the sweep, 64 (one row per lane) to 16384 rows (chunked
    partitions of 4096-row tiles), on a ragged 300_007-row system."""
    torch, cn = gpu
    n = 300_007
    log("partition", T, M)
    a, b, c, d = workloads.random_system(n, 77, "herm")
    ref = oracle_mod.thomas(a, b, c, d)
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    L = cn.Layout.contiguous(n, 1, partition=T, rows_per_thread=M)
    log("plan", cn.describe_plan(L))
    x = cn.solve(ta, tb, tc, td, layout=L)
    assert rel(x.cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("T", [8192, 16384])
def test_chunked_partitions_batch_and_short(gpu, oracle_mod, T):
    """Chunked partitions on a strided uniform batch whose systems end inside a partition's
    first chunk (5000 rows) or span several partitions (3 T + 11 rows), and in place."""
    torch, cn = gpu
    for n, batch in ((5000, 3), (3 * T + 11, 2)):
        a, b, c, d = workloads.random_system(n * batch, 13 + n % 7, "dd")
        ta, tb, tc, td = to_dev(torch, a, b, c, d)
        L = cn.Layout.contiguous(n, batch, partition=T)
        assert "chunks" in cn.describe_plan(L)
        cn.solve(ta, tb, tc, td, out=td, layout=L)
        got = td.cpu().numpy()
        for s_ in range(batch):
            sl = slice(s_ * n, (s_ + 1) * n)
            assert rel(got[sl], oracle_mod.thomas(a[sl], b[sl], c[sl], d[sl])) <= TOL


def test_plan_log_on_stderr(gpu):
    """CN_LOG=1: a new plan is described on stderr when it is built (a child process, since the
    library reads the variable once)."""
    import os
    import subprocess
    import sys

    code = ("import torch, paper_2205_00856_amd as cn; "
            "d = torch.ones(5000, dtype=torch.complex128, device='cuda'); "
            "a = 4 * d; cn.solve(a, d, d, d); torch.cuda.synchronize()")
    env = dict(os.environ, CN_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=240, cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert r.returncode == 0, r.stderr[-2000:]
    assert "cntri: plan for source 0, layout n=5000 batch=1" in r.stderr


def test_solve_in_place(gpu, oracle_mod):
    torch, cn = gpu
    n = 70_001
    a, b, c, d = workloads.random_system(n, 5, "dd")
    ref = oracle_mod.thomas(a, b, c, d)
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    cn.solve(ta, tb, tc, td, out=td)
    assert rel(td.cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("n,batch", [(300, 37), (5000, 9), (4096, 70), (1, 5), (129, 64)])
def test_solve_batched_contiguous(gpu, oracle_mod, n, batch):
    torch, cn = gpu
    log("batched", n, batch)
    a, b, c, d = workloads.random_system(n * batch, 3 + n, "herm")
    offs = np.arange(batch + 1) * n
    ref = oracle_mod.thomas_batched(offs, a, b, c, d, nthreads=8)
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    x = cn.solve(ta, tb, tc, td, layout=cn.Layout.contiguous(n, batch))
    assert rel(x.cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("n,batch", [(777, 50), (4096, 64), (6000, 3)])
def test_solve_interleaved(gpu, oracle_mod, n, batch):
    torch, cn = gpu
    log("interleaved", n, batch)
    a, b, c, d = workloads.random_system(n * batch, 11, "dd")
    # element (s, i) at i*batch + s: systems interleaved
    A, B, C, D = (v.reshape(n, batch) for v in (a, b, c, d))
    ref = np.empty((n, batch), np.complex128)
    for s in range(batch):
        ref[:, s] = oracle_mod.thomas(A[:, s], B[:, s], C[:, s], D[:, s])
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    x = cn.solve(ta, tb, tc, td, layout=cn.Layout.interleaved(n, batch))
    assert rel(x.cpu().numpy().reshape(n, batch), ref) <= TOL


def test_solve_uneven_batch(gpu, oracle_mod):
    torch, cn = gpu
    g = np.random.default_rng(8)
    lengths = np.concatenate([[1, 2, 4096, 4097, 0, 65_536], g.integers(1, 20_000, 40)])
    offs = np.concatenate([[0], np.cumsum(lengths)])
    a, b, c, d = workloads.random_system(int(offs[-1]), 21, "herm")
    ref = oracle_mod.thomas_batched(offs, a, b, c, d, nthreads=8)
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    x = cn.solve(ta, tb, tc, td, layout=cn.Layout.uneven(offs))
    assert rel(x.cpu().numpy(), ref) <= TOL


def test_solve_is_deterministic(gpu):
    torch, cn = gpu
    n = 500_000
    a, b, c, d = workloads.random_system(n, 2, "herm")
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    x1 = cn.solve(ta, tb, tc, td)
    x2 = cn.solve(ta, tb, tc, td)
    assert torch.equal(x1, x2)


def test_breakdown_flag(gpu):
    torch, cn = gpu
    n = 5000
    a, b, c, d = workloads.random_system(n, 2, "dd")
    a[1234] = 0.0
    b[1234] = 0.0
    c[1234] = 0.0  # exactly singular row
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    cn.solve(ta, tb, tc, td)
    assert cn.get_status() == 1
    assert cn.get_status() == 0  # the flag clears


def test_breakdown_flag_nan_rhs(gpu):
    """A NaN in d propagates to x; the status flag reports it and the call itself succeeds."""
    torch, cn = gpu
    a, b, c, d = workloads.random_system(3000, 4, "dd")
    d[1777] = np.nan
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    x = cn.solve(ta, tb, tc, td)
    assert not torch.isfinite(x).all()
    assert cn.get_status() == 1
    assert cn.get_status() == 0


@pytest.mark.parametrize("n,batch,es,bs", [(1000, 5, 3, 3100), (300, 6, 2, 700),
                                          (700, 70, 77, 1), (33, 64, 70, 1)])
def test_solve_strided_with_padding(gpu, oracle_mod, n, batch, es, bs):
    """Row stride > 1 with gaps between systems, and interleaved systems with padding columns;
    the padding elements must stay untouched."""
    torch, cn = gpu
    log("strided", n, batch, es, bs)
    span = (batch - 1) * bs + (n - 1) * es + 1
    rng = np.random.default_rng(n + es)
    a, b, c, d = workloads.random_system(n * batch, 40 + n, "herm")
    idx = (np.arange(batch)[:, None] * bs + np.arange(n)[None, :] * es).ravel()
    bufs = []
    for v in (a, b, c, d):
        full = workloads.complex_normal(rng, span)
        full[idx] = v
        bufs.append(full)
    offs = np.arange(batch + 1) * n
    ref = oracle_mod.thomas_batched(offs, a, b, c, d, nthreads=8)
    ta, tb, tc, td = to_dev(torch, *bufs)
    x0 = workloads.complex_normal(rng, span)
    tx = to_dev(torch, x0)[0]
    L = cn.Layout(n=n, batch=batch, elem_stride=es, batch_stride=bs)
    cn.solve(ta, tb, tc, td, out=tx, layout=L)
    out = tx.cpu().numpy()
    assert rel(out[idx], ref) <= TOL
    pad = np.setdiff1d(np.arange(span), idx)
    assert np.array_equal(out[pad], x0[pad])


def test_capture_without_reserve_is_refused(gpu):
    """A layout whose plan or workspace does not exist yet cannot be used inside a graph
    capture: the call returns CN_ERR_NOT_RESERVED and launches nothing."""
    torch, cn = gpu
    from paper_2205_00856_amd import _lib

    n = 12_345  # a layout no other test plans
    rng = np.random.default_rng(5)
    psi = to_dev(torch, workloads.complex_normal(rng, n))[0]
    V = to_dev(torch, rng.uniform(-1, 0, n))[0]
    out = torch.empty_like(psi)
    side = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    err = None
    try:
        with torch.cuda.graph(g, stream=side):
            cn.step(psi, V, 0.1, 0.01, out=out, layout=cn.Layout.contiguous(n, 1))
    except _lib.CnError as ex:
        err = ex
    except RuntimeError as ex:  # the capture context may wrap the library error
        err = ex
    assert err is not None and "NOT_RESERVED" in str(err)
    torch.cuda.synchronize()
    # after cn.reserve the same call captures and replays
    cn.reserve(cn.Layout.contiguous(n, 1))
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2, stream=side):
        cn.step(psi, V, 0.1, 0.01, out=out, layout=cn.Layout.contiguous(n, 1))
    g2.replay()
    torch.cuda.synchronize()
    ref = cn.step(psi, V, 0.1, 0.01, layout=cn.Layout.contiguous(n, 1))
    assert torch.equal(out, ref)


# ------------------------------------------------------------------ assembly, rhs, step
@pytest.mark.parametrize("field", [False, True])
def test_assemble_and_rhs(gpu, oracle_mod, field):
    torch, cn = gpu
    n, dx, dt = 3001, 0.07, 0.013
    inp = workloads.random_cn(n, 4, dx, dt)
    xg = workloads.grid_1d(n, dx) if field else None
    E = 0.21 if field else 0.0
    a0, b0, c0 = oracle_mod.cn_coeffs(inp["V"], dx, dt, xg, E)
    d0 = oracle_mod.cn_rhs(inp["psi"], inp["V"], dx, dt, xg, E)
    tV, tpsi = to_dev(torch, inp["V"], inp["psi"])
    txg = to_dev(torch, xg)[0] if field else None
    a, b, c = cn.assemble(tV, dx, dt, E=E, xgrid=txg)
    d = cn.rhs(tpsi, tV, dx, dt, E=E, xgrid=txg)
    for g, r in ((a, a0), (b, b0), (c, c0), (d, d0)):
        assert rel(g.cpu().numpy(), r) <= 1e-14


@pytest.mark.parametrize("n", [1, 2, 100, 4096, 4097, 65_536, 100_003, 1 << 20, 2_100_003])
def test_cn_step(gpu, oracle_mod, n):
    torch, cn = gpu
    log("cn_step", n)
    inp = workloads.random_cn(n, 31 + n, 0.1, 0.02)
    ref = oracle_mod.cn_step(inp["psi"], inp["V"], 0.1, 0.02)
    tV, tpsi = to_dev(torch, inp["V"], inp["psi"])
    out = cn.step(tpsi, tV, 0.1, 0.02)
    assert rel(out.cpu().numpy(), ref) <= TOL
    cn.step(tpsi, tV, 0.1, 0.02, out=tpsi)  # in place, multi-tile halos
    assert rel(tpsi.cpu().numpy(), ref) <= TOL


def test_cn_step_field_and_scale(gpu, oracle_mod):
    torch, cn = gpu
    n, dx, dt, E = 200_000, 0.05, 0.01, 0.037
    inp = workloads.random_cn(n, 9, dx, dt)
    xg = workloads.grid_1d(n, dx)
    ref = oracle_mod.cn_step(inp["psi"], 0.5 * inp["V"], dx, dt, xg, E)
    tV, tpsi, txg = to_dev(torch, inp["V"], inp["psi"], xg)
    out = cn.step(tpsi, tV, dx, dt, E=E, xgrid=txg, v_scale=0.5)
    assert rel(out.cpu().numpy(), ref) <= TOL


def test_plain_1d_one_solve_and_200_steps(gpu, oracle_mod):
    """The plain 1D workload: one materialised solve, then 200 chained steps."""
    torch, cn = gpu
    w = workloads.plain_1d()
    a0, b0, c0 = oracle_mod.cn_coeffs(w["V"], w["dx"], w["dt"])
    d0 = oracle_mod.cn_rhs(w["psi0"], w["V"], w["dx"], w["dt"])
    x0 = oracle_mod.thomas(a0, b0, c0, d0)
    ref = oracle_mod.cn_propagate(w["psi0"], w["V"], w["dx"], w["dt"], w["steps"])
    tV, tpsi = to_dev(torch, w["V"], w["psi0"])
    a, b, c = cn.assemble(tV, w["dx"], w["dt"])
    d = cn.rhs(tpsi, tV, w["dx"], w["dt"])
    x = cn.solve(a, b, c, d)
    assert rel(x.cpu().numpy(), x0) <= TOL
    cn.propagate(tpsi, tV, w["dx"], w["dt"], w["steps"])
    out = tpsi.cpu().numpy()
    assert rel(out, ref) <= TOL
    norm0 = np.sum(np.abs(w["psi0"]) ** 2) * w["dx"]
    assert abs(np.sum(np.abs(out) ** 2) * w["dx"] - norm0) <= 1e-11


def test_cn_step_uneven_batch(gpu, oracle_mod):
    torch, cn = gpu
    wl = workloads.uneven_batch(batch=300, hi=20_000, steps=1, seed=5)
    ref = oracle_mod.cn_step_batched(wl["offsets"], wl["psi0"], wl["V"], wl["dx"], wl["dt"], 8)
    tV, tpsi, tdx = to_dev(torch, wl["V"], wl["psi0"], wl["dx"])
    out = cn.step(tpsi, tV, 0.0, wl["dt"], dx_per_system=tdx,
                  layout=cn.Layout.uneven(wl["offsets"]))
    assert rel(out.cpu().numpy(), ref) <= TOL


def test_adi_step_small(gpu, oracle_mod):
    """Lie-split ADI step: x-lines (contiguous) then y-lines (interleaved), V/2 each."""
    torch, cn = gpu
    w = workloads.adi_2d(n=256, steps=3)
    ny, nx = w["psi0"].shape
    ref = w["psi0"]
    for _ in range(w["steps"]):
        ref = oracle_mod.adi_step(ref, w["V"], w["dx"], w["dy"], w["dt"], 8)
    tV, tpsi = to_dev(torch, w["V"].ravel(), w["psi0"].ravel())
    Lx = cn.Layout.contiguous(nx, ny)
    Ly = cn.Layout.interleaved(ny, nx)
    for _ in range(w["steps"]):
        cn.step(tpsi, tV, w["dx"], w["dt"], v_scale=0.5, out=tpsi, layout=Lx)
        cn.step(tpsi, tV, w["dy"], w["dt"], v_scale=0.5, out=tpsi, layout=Ly)
    assert rel(tpsi.cpu().numpy().reshape(ny, nx), ref) <= TOL


# ------------------------------------------------------------------ uniform batches of CN steps
# Contiguous CN steps of many systems of 1024 < n <= 4096 (whole systems in one workgroup, the
# ADI x-sweep path): per-system dx, ragged n (whole lane blocks past the end at n = 1032, 4000),
# in place, and V 8 bytes off a 16-byte boundary.
@pytest.mark.parametrize("n,batch", [(4096, 600), (2048, 1100), (1032, 1030), (4000, 520)])
def test_cn_step_uniform_batch(gpu, oracle_mod, n, batch):
    torch, cn = gpu
    log("cn_step uniform batch", n, batch)
    dt = 0.02
    rng = np.random.default_rng(1234 + n)
    psi = workloads.complex_normal(rng, n * batch)
    V = rng.uniform(-2.0, 2.0, n * batch)
    dxs = rng.uniform(0.05, 0.2, batch)
    offs = np.arange(batch + 1, dtype=np.int64) * n
    ref = oracle_mod.cn_step_batched(offs, psi, V, dxs, dt, 8)
    L = cn.Layout.contiguous(n, batch)
    assert "single" in cn.describe_plan(L, cn_mode=True)
    tV, tpsi, tdx = to_dev(torch, V, psi, dxs)
    out = cn.step(tpsi, tV, 0.0, dt, dx_per_system=tdx, layout=L)
    assert rel(out.cpu().numpy(), ref) <= TOL
    cn.step(tpsi, tV, 0.0, dt, dx_per_system=tdx, out=tpsi, layout=L)  # in place
    assert torch.equal(tpsi, out)
    Vpad = torch.empty(n * batch + 1, dtype=torch.float64, device="cuda")
    Vpad[1:] = tV
    out2 = cn.step(to_dev(torch, psi)[0], Vpad[1:], 0.0, dt, dx_per_system=tdx, layout=L)
    assert rel(out2.cpu().numpy(), ref) <= TOL


# Interior wavefronts (every row and both halo rows inside the system) run a second compiled
# path without clamps or edge selects.  In a 4096-row tile (8 wavefronts of 512 rows) the last
# wavefront turns interior at n = 3585; the sizes straddle that and the first wavefront's edge,
# for the fused CN step and for the explicit solve (single tile and two-pass tiles).
@pytest.mark.parametrize("n", [3584, 3585, 3586, 4095, 4096])
def test_interior_wavefront_boundary_cn(gpu, oracle_mod, n):
    torch, cn = gpu
    log("interior boundary cn", n)
    batch, dt = 64, 0.02
    rng = np.random.default_rng(77 + n)
    psi = workloads.complex_normal(rng, n * batch)
    V = rng.uniform(-2.0, 2.0, n * batch)
    dxs = rng.uniform(0.05, 0.2, batch)
    offs = np.arange(batch + 1, dtype=np.int64) * n
    ref = oracle_mod.cn_step_batched(offs, psi, V, dxs, dt, 8)
    tV, tpsi, tdx = to_dev(torch, V, psi, dxs)
    out = cn.step(tpsi, tV, 0.0, dt, dx_per_system=tdx, layout=cn.Layout.contiguous(n, batch))
    assert rel(out.cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("n,T,M", [(3585, 4096, 8), (3584, 4096, 8), (5 * 1024 + 1, 1024, 4),
                                   (5 * 1024 - 1, 1024, 4), (2048 + 257, 2048, 8)])
def test_interior_wavefront_boundary_solve(gpu, oracle_mod, n, T, M):
    torch, cn = gpu
    log("interior boundary solve", n, T, M)
    a, b, c, d = workloads.random_system(n, 300 + n, "herm")
    ref = oracle_mod.thomas(a, b, c, d)
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    x = cn.solve(ta, tb, tc, td, layout=cn.Layout.contiguous(n, 1, partition=T, rows_per_thread=M))
    assert rel(x.cpu().numpy(), ref) <= TOL


def test_cn_step_uniform_batch_repeated(gpu, oracle_mod):
    """Five chained in-place steps of 4096 x 4096 rows at one dx (the ADI x-sweep shape at
    half the lines), against the oracle stepping each line."""
    torch, cn = gpu
    n, batch, dx, dt = 4096, 2048, 0.1, 0.01
    rng = np.random.default_rng(99)
    psi = workloads.complex_normal(rng, n * batch)
    V = rng.uniform(0.0, 5.0, n * batch)
    offs = np.arange(batch + 1, dtype=np.int64) * n
    ref = psi
    for _ in range(5):
        ref = oracle_mod.cn_step_batched(offs, ref, V, np.full(batch, dx), dt, 8)
    L = cn.Layout.contiguous(n, batch)
    tV, tpsi = to_dev(torch, V, psi)
    for _ in range(5):
        cn.step(tpsi, tV, dx, dt, out=tpsi, layout=L)
    assert rel(tpsi.cpu().numpy(), ref) <= TOL


# ------------------------------------------------------------------ adjoint
@pytest.mark.parametrize("n", [7, 4096, 100_001])
def test_solve_adjoint(gpu, oracle_mod, n):
    torch, cn = gpu
    a, b, c, d = workloads.random_system(n, 17, "dd")
    g = np.random.default_rng(3)
    G = g.standard_normal(n) + 1j * g.standard_normal(n)
    x = oracle_mod.thomas(a, b, c, d)
    lam, ga, gb, gc = oracle_mod.thomas_adjoint(a, b, c, x, G)
    ta, tb, tc, tx, tG = to_dev(torch, a, b, c, x, G)
    gd_, ga_, gb_, gc_ = cn.solve_adjoint(ta, tb, tc, tx, tG)
    assert rel(gd_.cpu().numpy(), lam) <= TOL
    assert rel(ga_.cpu().numpy(), ga) <= TOL
    assert rel(gb_.cpu().numpy(), gb) <= TOL
    assert rel(gc_.cpu().numpy(), gc) <= TOL


@pytest.mark.parametrize("n", [50, 5000, 300_001, 1 << 20])
def test_step_adjoint(gpu, oracle_mod, n):
    torch, cn = gpu
    dx, dt, E = 0.05, 0.01, 0.02
    inp = workloads.random_cn(n, 12, dx, dt)
    xg = workloads.grid_1d(n, dx)
    g = np.random.default_rng(4)
    G1 = g.standard_normal(n) + 1j * g.standard_normal(n)
    p1 = oracle_mod.cn_step(inp["psi"], inp["V"], dx, dt, xg, E)
    g0, dV, dE = oracle_mod.cn_propagate_grad(inp["psi"], inp["V"], dx, dt, 1, G1, xg, [E])
    tV, tp0, tp1, tG, txg = to_dev(torch, inp["V"], inp["psi"], p1, G1, xg)
    tdV = torch.zeros(n, dtype=torch.float64, device="cuda")
    tdE = torch.zeros(1, dtype=torch.float64, device="cuda")
    gn = cn.step_adjoint(tp0, tp1, tG, tV, dx, dt, E=E, xgrid=txg, dV=tdV, dE_out=tdE)
    assert rel(gn.cpu().numpy(), g0) <= TOL
    assert rel(tdV.cpu().numpy(), dV) <= TOL
    assert abs(tdE.cpu().numpy()[0] - dE[0]) <= TOL * max(abs(dE[0]), 1e-300) + 1e-13


# ------------------------------------------------------------------ hipGraph capture
def test_graph_captured_adi_step_replays(gpu, oracle_mod):
    """One ADI step captured as a graph, replayed several times with eager work and
    synchronisations in between; every replay matches the eager result bit for bit."""
    torch, cn = gpu
    w = workloads.adi_2d(n=512, steps=1, seed=77)
    ny, nx = w["psi0"].shape
    tV, p0 = to_dev(torch, w["V"].ravel(), w["psi0"].ravel())
    Lx = cn.Layout.contiguous(nx, ny)
    Ly = cn.Layout.interleaved(ny, nx)
    cn.reserve(Lx)
    cn.reserve(Ly)
    psi = p0.clone()

    def step(p):
        cn.step(p, tV, w["dx"], w["dt"], v_scale=0.5, out=p, layout=Lx)
        cn.step(p, tV, w["dy"], w["dt"], v_scale=0.5, out=p, layout=Ly)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step(psi)
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step(psi)
    ref = oracle_mod.adi_step(w["psi0"], w["V"], w["dx"], w["dy"], w["dt"], 8)
    eager = p0.clone()
    step(eager)
    assert rel(eager.cpu().numpy().reshape(ny, nx), ref) <= TOL
    for _ in range(4):
        psi.copy_(p0)
        g.replay()
        torch.cuda.synchronize()
        junk = p0.clone()
        step(junk)  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(psi, eager)


def test_propagate_adjoint_overlapped_equals_captured(gpu):
    """Reverse mode run eagerly (the recompute of the next segment overlapped on a second
    stream) and replayed from a graph capture (segments one after the other on the captured
    stream) give the same bits for g, dV and dE; eager work runs between the replays."""
    torch, cn = gpu
    n, dx, dt, steps, K = 50_000, 0.05, 0.01, 23, 5
    rng = np.random.default_rng(21)
    x = workloads.grid_1d(n, dx)
    V = workloads.softcore(x)
    E = rng.normal(0, 0.05, steps)
    tV, tx, tpsi = to_dev(torch, V, x, workloads.gaussian(x, 0.0, 5.0, 1.0, dx))
    gT = to_dev(torch, workloads.complex_normal(rng, n))[0]
    L = cn.Layout.contiguous(n, 1)
    ckpt = torch.empty(((steps + K - 1) // K) * n, dtype=torch.complex128, device="cuda")
    cn.propagate(tpsi.clone(), tV, dx, dt, steps, E=E, xgrid=tx, ckpt=ckpt, K=K, layout=L)
    seg = torch.empty((K + 1) * n, dtype=torch.complex128, device="cuda")

    def fresh():
        return (gT.clone(), torch.zeros(n, dtype=torch.float64, device="cuda"),
                torch.zeros(steps, dtype=torch.float64, device="cuda"))

    def run(g, dV, dE):
        cn.propagate_adjoint(ckpt, g, tV, dx, dt, steps, K, E=E, xgrid=tx, dV=dV, dE=dE,
                             seg=seg, layout=L)

    ge, dVe, dEe = fresh()
    run(ge, dVe, dEe)
    torch.cuda.synchronize()
    gc, dVc, dEc = fresh()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        run(gc, dVc, dEc)
    for _ in range(3):
        gc.copy_(gT)
        dVc.zero_()
        dEc.zero_()
        graph.replay()
        torch.cuda.synchronize()
        run(*fresh())  # eager work between the replays
        torch.cuda.synchronize()
        assert torch.equal(gc, ge) and torch.equal(dVc, dVe) and torch.equal(dEc, dEe)


# ------------------------------------------------------------------ persistent uneven launch
@pytest.mark.parametrize("partition", [1024, 0])
def test_uneven_repeated_steps(gpu, oracle_mod, partition):
    """Three chained in-place steps: one persistent launch each (partition 1024; its device
    queue resets itself), or the automatic per-length launches with two-pass long systems."""
    torch, cn = gpu
    wl = workloads.uneven_batch(batch=500, lo=1, hi=65_536, steps=3, seed=9)
    offs, dt = wl["offsets"], wl["dt"]
    ref = wl["psi0"]
    for _ in range(3):
        ref = oracle_mod.cn_step_batched(offs, ref, wl["V"], wl["dx"], dt, 8)
    tV, tpsi, tdx = to_dev(torch, wl["V"], wl["psi0"], wl["dx"])
    L = cn.Layout.uneven(offs, partition=partition, rows_per_thread=4 if partition else 0)
    plan = cn.describe_plan(L, True)
    assert ("persistent" in plan) == (partition > 0), plan
    for _ in range(3):
        cn.step(tpsi, tV, 0.0, dt, dx_per_system=tdx, out=tpsi, layout=L)
    assert rel(tpsi.cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("T,M", [(512, 4), (1024, 4), (2048, 4), (1024, 8), (2048, 8)])
def test_uneven_persistent_configs_and_long_fallback(gpu, oracle_mod, T, M):
    torch, cn = gpu
    g = np.random.default_rng(T + M)
    # one system longer than 64 tiles takes the multi-workgroup path in the same call
    lengths = np.concatenate([[64 * T + 17, 3, 0, 1], g.integers(1, 64 * T, 60)])
    offs = np.concatenate([[0], np.cumsum(lengths)])
    a, b, c, d = workloads.random_system(int(offs[-1]), 5, "herm")
    ref = oracle_mod.thomas_batched(offs, a, b, c, d, nthreads=8)
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    L = cn.Layout.uneven(offs, partition=T, rows_per_thread=M)
    # the multi-workgroup launch and its reduced system cover the long system only
    K = (64 * T + 17 + T - 1) // T
    assert f"systems=1 tiles={K};" in cn.describe_plan(L)
    x = cn.solve(ta, tb, tc, td, layout=L)
    assert rel(x.cpu().numpy(), ref) <= TOL
    assert cn.get_status() == 0
    gx = torch.ones_like(td)
    lam, _, _, _ = cn.solve_adjoint(ta, tb, tc, x, gx, need_abc=False, layout=L)
    lam_ref = np.concatenate([
        oracle_mod.thomas_adjoint(a[o0:o1], b[o0:o1], c[o0:o1], ref[o0:o1],
                                  np.ones(o1 - o0, complex))[0]
        for o0, o1 in zip(offs[:-1], offs[1:]) if o1 > o0])
    assert rel(lam.cpu().numpy(), lam_ref) <= TOL
    assert cn.get_status() == 0


def test_autotune_keeps_results(gpu, oracle_mod):
    torch, cn = gpu
    wl = workloads.uneven_batch(batch=200, hi=30_000, steps=1, seed=12)
    ref = oracle_mod.cn_step_batched(wl["offsets"], wl["psi0"], wl["V"], wl["dx"], wl["dt"], 8)
    tV, tpsi, tdx = to_dev(torch, wl["V"], wl["psi0"], wl["dx"])
    L = cn.Layout.uneven(wl["offsets"])
    out = torch.empty_like(tpsi)
    rep = cn.autotune(L, tpsi, out, V=tV, dt=wl["dt"], dx_per_system=tdx)
    log(rep)
    assert "chosen" in rep and "automatic" in rep
    out2 = cn.step(tpsi, tV, 0.0, wl["dt"], dx_per_system=tdx, layout=L)
    assert rel(out2.cpu().numpy(), ref) <= TOL
    # a sequence over the tuned plan (fused when it has a two-pass group)
    ref3 = wl["psi0"]
    for _ in range(3):
        ref3 = oracle_mod.cn_step_batched(wl["offsets"], ref3, wl["V"], wl["dx"], wl["dt"], 8)
    p3 = tpsi.clone()
    cn.propagate(p3, tV, 0.0, wl["dt"], 3, dx_per_system=tdx, layout=L)
    assert rel(p3.cpu().numpy(), ref3) <= TOL
    # a long CN line tuned in cn_step mode, then propagated
    m, dxm, dtm = 300_001, 0.1, 0.02
    inp = workloads.random_cn(m, 44, dxm, dtm)
    mV, mp = to_dev(torch, inp["V"], inp["psi"])
    Lm = cn.Layout.contiguous(m, 1)
    rep = cn.autotune(Lm, mp, torch.empty_like(mp), V=mV, dx=dxm, dt=dtm)
    log(rep)
    cn.propagate(mp, mV, dxm, dtm, 4, layout=Lm)
    assert rel(mp.cpu().numpy(), oracle_mod.cn_propagate(inp["psi"], inp["V"], dxm, dtm, 4)) <= TOL
    n = 200_000
    a, b, c, d = workloads.random_system(n, 3, "dd")
    xref = oracle_mod.thomas(a, b, c, d)
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    x = torch.empty_like(td)
    rep = cn.autotune(cn.Layout.contiguous(n, 1), td, x, a=ta, b=tb, c=tc)
    log(rep)
    x2 = cn.solve(ta, tb, tc, td)
    assert rel(x2.cpu().numpy(), xref) <= TOL


# ------------------------------------------------------------------ interleaved (column) kernels
@pytest.mark.parametrize("T,M", [(64, 8), (64, 4), (64, 16), (128, 8)])
@pytest.mark.parametrize("n,batch", [(1000, 70), (4096, 128), (33, 64)])
def test_column_kernels(gpu, oracle_mod, T, M, n, batch):
    torch, cn = gpu
    log("columns", T, M, n, batch)
    a, b, c, d = workloads.random_system(n * batch, 7 + n, "herm")
    A, B, C, D = (v.reshape(n, batch) for v in (a, b, c, d))
    ref = np.empty((n, batch), np.complex128)
    lam_ref = np.empty((n, batch), np.complex128)
    for s in range(batch):
        ref[:, s] = oracle_mod.thomas(A[:, s], B[:, s], C[:, s], D[:, s])
        lam_ref[:, s] = oracle_mod.thomas_adjoint(A[:, s], B[:, s], C[:, s], ref[:, s], D[:, s])[0]
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    L = cn.Layout.interleaved(n, batch, partition=T, rows_per_thread=M)
    assert "columns" in cn.describe_plan(L)
    x = cn.solve(ta, tb, tc, td, layout=L)
    assert rel(x.cpu().numpy().reshape(n, batch), ref) <= TOL
    tx = to_dev(torch, ref.ravel())[0]
    lam, _, _, _ = cn.solve_adjoint(ta, tb, tc, tx, td, need_abc=False, layout=L)
    assert rel(lam.cpu().numpy().reshape(n, batch), lam_ref) <= TOL
    # CN step in place on the interleaved layout (multi-tile halos)
    g = np.random.default_rng(n)
    V = g.uniform(-1, 0, (n, batch))
    psi = g.standard_normal((n, batch)) + 1j * g.standard_normal((n, batch))
    pref = np.empty_like(psi)
    for s in range(batch):
        pref[:, s] = oracle_mod.cn_step(psi[:, s], V[:, s], 0.1, 0.02)
    tV, tp = to_dev(torch, V.ravel(), psi.ravel())
    cn.step(tp, tV, 0.1, 0.02, out=tp, layout=L)
    assert rel(tp.cpu().numpy().reshape(n, batch), pref) <= TOL


# ------------------------------------------------------ nesting depth fixed by the caller
@pytest.mark.parametrize("n,T,M,levels", [(300_007, 1024, 4, 1), (300_007, 1024, 4, 2),
                                          (3_000_017, 128, 2, 1), (3_000_017, 128, 2, 2),
                                          (3_000_017, 128, 2, 3), (5, 128, 2, 1)])
def test_solve_with_fixed_levels(gpu, oracle_mod, n, T, M, levels):
    """cn_layout.levels = L: L partition levels, then the serial RS stage on what is left."""
    torch, cn = gpu
    log("levels", n, T, M, levels)
    a, b, c, d = workloads.random_system(n, 90 + levels, "herm")
    ref = oracle_mod.thomas(a, b, c, d)
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    L = cn.Layout.contiguous(n, 1, partition=T, rows_per_thread=M, levels=levels)
    plan = cn.describe_plan(L)
    if n > T:
        assert plan.count("multi") <= levels
    x = cn.solve(ta, tb, tc, td, layout=L)
    assert rel(x.cpu().numpy(), ref) <= TOL
    assert cn.get_status() == 0


def test_fixed_levels_batches_and_propagation(gpu, oracle_mod):
    """The serial RS stage on the reduced systems of a uniform batch (one thread each), of an
    uneven batch, and inside fused propagation (its rows take the deferred joint-row term)."""
    torch, cn = gpu
    n, batch = 20_000, 7
    a, b, c, d = workloads.random_system(n * batch, 5, "dd")
    offs = np.arange(batch + 1) * n
    ref = oracle_mod.thomas_batched(offs, a, b, c, d, nthreads=8)
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    L = cn.Layout.contiguous(n, batch, partition=512, levels=1)
    assert "serial RS" in cn.describe_plan(L)
    assert rel(cn.solve(ta, tb, tc, td, layout=L).cpu().numpy(), ref) <= TOL
    lengths = np.array([5000, 1, 0, 9000, 17_000])
    uo = np.concatenate([[0], np.cumsum(lengths)])
    a, b, c, d = workloads.random_system(int(uo[-1]), 6, "herm")
    ref = oracle_mod.thomas_batched(uo, a, b, c, d, nthreads=8)
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    Lu = cn.Layout.uneven(uo, levels=1)
    assert "serial RS" in cn.describe_plan(Lu)
    assert rel(cn.solve(ta, tb, tc, td, layout=Lu).cpu().numpy(), ref) <= TOL
    # propagation with a field: the fused chain with the serial RS stage as its reduced system
    w = workloads.differentiated(n=100_003, steps=12)
    refp = oracle_mod.cn_propagate(w["psi0"], w["V"], w["dx"], w["dt"], 12, w["x"], w["E"])
    tV, tp, tx = to_dev(torch, w["V"], w["psi0"], w["x"])
    Lp = cn.Layout.contiguous(w["n"], 1, levels=1)
    assert "serial RS" in cn.describe_plan(Lp, True)
    cn.propagate(tp, tV, w["dx"], w["dt"], 12, E=w["E"], xgrid=tx, layout=Lp)
    assert rel(tp.cpu().numpy(), refp) <= TOL
    assert cn.get_status() == 0


def test_plan_log_reports_stage_times(gpu):
    torch, cn = gpu
    n = 1_000_003
    a, b, c, d = workloads.random_system(n, 3, "herm")
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    L = cn.Layout.contiguous(n, 1, partition=1024, rows_per_thread=4, levels=1)
    cn.solve(ta, tb, tc, td, layout=L)
    cn.profile(True)
    cn.solve(ta, tb, tc, td, layout=L)
    cn.profile(False)
    rep = cn.profile_report()
    labels = [r[0] for r in rep]
    assert [lab.split()[1] for lab in labels] == ["reduce", "serial-RS", "subst"]
    assert all(ms > 0 for _, ms in rep)
    cn.solve(ta, tb, tc, td, layout=L)
    assert cn.profile_report() == []  # off: nothing logged


def test_autotune_cache_file(gpu, oracle_mod, tmp_path):
    """cn_autotune writes its choice to the persistent cache (a JSON file keyed by the layout's
    class); a fresh handle that reads the file plans the automatic layout with the cached
    configuration, and its results stay the oracle's."""
    torch, cn = gpu
    import ctypes
    import json

    from paper_2205_00856_amd import _lib

    path = str(tmp_path / "tune.json")
    n = 200_003
    a, b, c, d = workloads.random_system(n, 31, "herm")
    ref = oracle_mod.thomas(a, b, c, d)
    ta, tb, tc, td = to_dev(torch, a, b, c, d)
    L = cn.Layout.contiguous(n, 1)
    lib = _lib.lib()
    h = ctypes.c_void_p()
    assert lib.cn_create(ctypes.byref(h), 0) == _lib.CN_OK
    try:
        assert lib.cn_tune_cache(h, path.encode()) == _lib.CN_OK
        out = torch.empty_like(td)
        buf = ctypes.create_string_buffer(4096)
        Lc = L.c()
        st = lib.cn_autotune(h, ctypes.byref(Lc), 0, None, 0.0, ctypes.c_void_p(ta.data_ptr()),
                             ctypes.c_void_p(tb.data_ptr()), ctypes.c_void_p(tc.data_ptr()),
                             ctypes.c_void_p(td.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                             buf, 4096, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == _lib.CN_OK
        log(buf.value.decode())
        assert "(cached)" in buf.value.decode()
    finally:
        torch.cuda.synchronize()
        lib.cn_destroy(h)
    entries = json.load(open(path))
    (cls, ent), = entries.items()
    assert cls.startswith("gfx") and "|src0|uniform|n2^17|" in cls
    assert set(ent) == {"partition", "rows_per_thread", "ms"}
    # a fresh handle with the cache: the automatic layout takes the cached configuration
    h2 = ctypes.c_void_p()
    assert lib.cn_create(ctypes.byref(h2), 0) == _lib.CN_OK
    try:
        assert lib.cn_tune_cache(h2, path.encode()) == _lib.CN_OK
        Lc = L.c()
        assert lib.cn_describe_plan(h2, ctypes.byref(Lc), 0, buf, 4096) == _lib.CN_OK
        desc = buf.value.decode()
        if ent["partition"] > 0:
            assert f"T={ent['partition']}(M={ent['rows_per_thread']}" in desc
        x = torch.empty_like(td)
        st = lib.cn_tridiag_solve(h2, ctypes.byref(Lc), ctypes.c_void_p(ta.data_ptr()),
                                  ctypes.c_void_p(tb.data_ptr()), ctypes.c_void_p(tc.data_ptr()),
                                  ctypes.c_void_p(td.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == _lib.CN_OK
        torch.cuda.synchronize()
        assert rel(x.cpu().numpy(), ref) <= TOL
        # a hand-written entry for the same class is honoured as well
        with open(path, "w") as f:
            json.dump({cls: {"partition": 256, "rows_per_thread": 4, "ms": -1}}, f)
        assert lib.cn_tune_cache(h2, path.encode()) == _lib.CN_OK
        L2 = cn.Layout.contiguous(n + 1, 1).c()  # same class, a plan not built yet
        assert lib.cn_describe_plan(h2, ctypes.byref(L2), 0, buf, 4096) == _lib.CN_OK
        assert "T=256(M=4" in buf.value.decode()
    finally:
        torch.cuda.synchronize()
        lib.cn_destroy(h2)


def test_reserve_leaves_no_hip_error(gpu):
    """cn_reserve builds the plans of every source for a layout; for sources without kernels of
    a launch form (the column-only field coupling on an uneven batch with an explicit partition)
    it must refuse the plan without leaving a HIP error behind, which the caller's next kernel
    launch would report.  Same for an autotune run whose candidates include refused ones."""
    torch, cn = gpu
    import ctypes

    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipPeekAtLastError.restype = ctypes.c_int
    hip.hipGetLastError()  # start from a clean error state
    offs = np.cumsum([0, 3000, 70_000, 500, 9000]).astype(np.int64)
    cn.reserve(cn.Layout.uneven(offs, partition=1024, rows_per_thread=4))
    assert hip.hipPeekAtLastError() == 0
    t = torch.ones(1000, device="cuda").sum().item()  # a launch of the caller's after the call
    assert t == 1000.0
