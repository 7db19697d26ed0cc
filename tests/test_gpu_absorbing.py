"""GPU parity of the Crank-Nicolson step with an absorbing potential (the potential is V - iW,
so H is non-Hermitian and the explicit side 1 - i tau H is not T^dagger), against the CPU
oracle: the materialised coefficients and right-hand side, single steps on one system, uniform
and uneven batches, a propagation with a field and checkpoints, a captured graph, and the
entry points that refuse it.

Tolerance: relative L2 <= 1e-11 for states (FP64 on both sides; rounding only), 1e-13 for the
materialised coefficients and right-hand side (a few roundings per element).
"""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
TOL = 1e-11
UNSUPPORTED = -2


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


def case(n, seed, dx=0.1, dt=0.02):
    inp = workloads.random_cn(n, seed, dx, dt)
    W = workloads.absorber(n, 0.2, 3.0)
    return inp["V"], inp["psi"], W


@pytest.mark.parametrize("n", [1, 2, 37, 4096 + 17, 65_536, (1 << 20) + 3])
def test_step_with_absorber(gpu, oracle_mod, n):
    torch, cn = gpu
    log("absorbing step", n)
    dx, dt = 0.1, 0.02
    V, psi, W = case(n, 60 + n % 97, dx, dt)
    ref = oracle_mod.cn_step(psi, V, dx, dt, W=W)
    tV, tpsi, tW = to_dev(torch, V, psi, W)
    out = cn.step(tpsi, tV, dx, dt, W=tW).cpu().numpy()
    assert rel(out, ref) <= TOL
    if n > 1:  # the absorber takes norm away
        assert np.sum(np.abs(out) ** 2) < np.sum(np.abs(psi) ** 2)
    assert cn.get_status() == 0


def test_assemble_and_rhs_with_absorber(gpu, oracle_mod):
    torch, cn = gpu
    n, dx, dt = 5000, 0.07, 0.03
    V, psi, W = case(n, 3, dx, dt)
    xg = workloads.grid_1d(n, dx)
    E = 0.21
    ra, rb, rc = oracle_mod.cn_coeffs(V, dx, dt, xg, E, W=W)
    rd = oracle_mod.cn_rhs(psi, V, dx, dt, xg, E, W=W)
    tV, tpsi, tW, txg = to_dev(torch, V, psi, W, xg)
    a, b, c = cn.assemble(tV, dx, dt, E=E, xgrid=txg, W=tW)
    d = cn.rhs(tpsi, tV, dx, dt, E=E, xgrid=txg, W=tW)
    for got, want in ((a, ra), (b, rb), (c, rc), (d, rd)):
        assert rel(got.cpu().numpy(), want) <= 1e-13
    assert np.max(np.abs(a.cpu().numpy().real - (1 + 0.5 * dt * W))) <= 1e-15


def test_zero_absorber_matches_hermitian_step(gpu):
    """W = 0 through the materialised path gives the fused Hermitian step up to rounding."""
    torch, cn = gpu
    n, dx, dt = 200_003, 0.1, 0.02
    V, psi, _ = case(n, 8, dx, dt)
    tV, tpsi = to_dev(torch, V, psi)
    tW = torch.zeros(n, dtype=torch.float64, device="cuda")
    a = cn.step(tpsi, tV, dx, dt, W=tW).cpu().numpy()
    b = cn.step(tpsi, tV, dx, dt).cpu().numpy()
    assert rel(a, b) <= 1e-13


def test_propagate_with_absorber_field_and_checkpoints(gpu, oracle_mod):
    """The absorbing workload (packet moving into the ramp at the right wall) with a field:
    60 steps against the oracle, the checkpoints against the oracle's states, and the norm
    falling step by step."""
    torch, cn = gpu
    w = workloads.absorbing_1d(n=65_536)
    steps, K = 60, 20
    E = np.random.default_rng(2).normal(0.0, 0.05, steps)
    log("absorbing propagate", steps)
    tV, tpsi, tW, txg = to_dev(torch, w["V"], w["psi0"], w["W"], w["x"])
    ckpt = torch.empty(steps // K * w["n"], dtype=torch.complex128, device="cuda")
    cn.propagate(tpsi, tV, w["dx"], w["dt"], steps, E=E, xgrid=txg, ckpt=ckpt, K=K, W=tW)
    ref = w["psi0"]
    ck = ckpt.cpu().numpy().reshape(steps // K, w["n"])
    for k in range(steps):
        if k % K == 0:
            assert rel(ck[k // K], ref) <= TOL
        ref = oracle_mod.cn_step(ref, w["V"], w["dx"], w["dt"], w["x"], E[k], W=w["W"])
    out = tpsi.cpu().numpy()
    assert rel(out, ref) <= TOL
    assert np.sum(np.abs(out) ** 2) < np.sum(np.abs(w["psi0"]) ** 2)


def test_propagate_with_absorber_no_field(gpu, oracle_mod):
    """Without a field T is assembled once and reused by every step."""
    torch, cn = gpu
    w = workloads.absorbing_1d(n=30_000)
    steps = 40
    ref = oracle_mod.cn_propagate(w["psi0"], w["V"], w["dx"], w["dt"], steps, W=w["W"])
    tV, tpsi, tW = to_dev(torch, w["V"], w["psi0"], w["W"])
    cn.propagate(tpsi, tV, w["dx"], w["dt"], steps, W=tW)
    assert rel(tpsi.cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("interleaved", [False, True])
def test_batched_step_with_absorber(gpu, oracle_mod, interleaved):
    torch, cn = gpu
    n, batch, dx, dt = 3001, 8, 0.1, 0.02
    g = np.random.default_rng(11)
    V = g.uniform(-1.0, 0.0, (batch, n))
    P = workloads.complex_normal(g, (batch, n))
    W = np.stack([workloads.absorber(n, 0.1 + 0.02 * s, 1.0 + s) for s in range(batch)])
    if interleaved:
        L = cn.Layout.interleaved(n, batch)
        tV, tP, tW = to_dev(torch, V.T.ravel(), P.T.ravel(), W.T.ravel())
    else:
        L = cn.Layout.contiguous(n, batch)
        tV, tP, tW = to_dev(torch, V.ravel(), P.ravel(), W.ravel())
    out = cn.step(tP, tV, dx, dt, W=tW, layout=L).cpu().numpy()
    out = out.reshape(n, batch).T if interleaved else out.reshape(batch, n)
    for s in range(batch):
        ref = oracle_mod.cn_step(P[s], V[s], dx, dt, W=W[s])
        assert rel(out[s], ref) <= TOL


def test_uneven_step_with_absorber(gpu, oracle_mod):
    torch, cn = gpu
    wl = workloads.uneven_batch(batch=200, hi=20_000, steps=1, seed=7)
    offs = wl["offsets"]
    W = np.concatenate([workloads.absorber(int(offs[s + 1] - offs[s]))
                        for s in range(wl["batch"])])
    tV, tpsi, tdx, tW = to_dev(torch, wl["V"], wl["psi0"], wl["dx"], W)
    out = cn.step(tpsi, tV, 0.0, wl["dt"], dx_per_system=tdx, W=tW,
                  layout=cn.Layout.uneven(offs)).cpu().numpy()
    for s in range(wl["batch"]):
        o0, o1 = offs[s], offs[s + 1]
        ref = oracle_mod.cn_step(wl["psi0"][o0:o1], wl["V"][o0:o1], wl["dx"][s], wl["dt"],
                                 W=W[o0:o1])
        assert rel(out[o0:o1], ref) <= TOL


def test_absorbing_step_graph_replays(gpu):
    """After one call outside capture (which sizes the handle's buffer), the materialised step
    captures; replays with eager work between them give the eager result bit for bit."""
    torch, cn = gpu
    n, dx, dt, steps = 100_001, 0.1, 0.02, 4
    V, psi, W = case(n, 31, dx, dt)
    tV, p0, tW = to_dev(torch, V, psi, W)
    L = cn.Layout.contiguous(n, 1)
    cn.reserve(L)
    eager = p0.clone()
    cn.propagate(eager, tV, dx, dt, steps, layout=L, W=tW)
    torch.cuda.synchronize()
    x = p0.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        cn.propagate(x, tV, dx, dt, steps, layout=L, W=tW)
    for _ in range(3):
        x.copy_(p0)
        graph.replay()
        torch.cuda.synchronize()
        junk = p0.clone()
        cn.step(junk, tV, dx, dt, out=junk, layout=L)
        torch.cuda.synchronize()
        assert torch.equal(x, eager)


def test_absorber_refusals(gpu):
    """The adjoint entry points, the autotuner and shared coefficients refuse the absorbing
    term with CN_ERR_UNSUPPORTED."""
    torch, cn = gpu
    from paper_2205_00856_amd import _lib
    from paper_2205_00856_amd.api import _operator

    n, dx, dt = 1000, 0.1, 0.02
    V, psi, W = case(n, 4, dx, dt)
    tV, tpsi, tW = to_dev(torch, V, psi, W)
    g = tpsi.clone()
    op = _operator(tV, dx, dt, W=tW)
    h = cn.handle(0)
    L = cn.Layout.contiguous(n, 1).c()
    lib = _lib.lib()
    st = lib.cn_step_adjoint(h.ptr, ctypes.byref(L), ctypes.byref(op), 0.0,
                             ctypes.c_void_p(tpsi.data_ptr()), ctypes.c_void_p(tpsi.data_ptr()),
                             ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                             None, None, None)
    assert st == UNSUPPORTED
    seg = torch.empty_like(tpsi)
    st = lib.cn_propagate_adjoint(h.ptr, ctypes.byref(L), ctypes.byref(op), 1, None,
                                  ctypes.c_void_p(tpsi.data_ptr()), 1,
                                  ctypes.c_void_p(seg.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                  None, None, None)
    assert st == UNSUPPORTED
    out = torch.empty_like(tpsi)
    st = lib.cn_autotune(h.ptr, ctypes.byref(L), 1, ctypes.byref(op), 0.0, None, None, None,
                         ctypes.c_void_p(tpsi.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                         None, 0, None)
    assert st == UNSUPPORTED
    Ls = cn.Layout.contiguous(n, 2, shared_coefficients=True)
    two = torch.cat([tpsi, tpsi])
    with pytest.raises(_lib.CnError):
        cn.step(two, tV, dx, dt, W=tW, layout=Ls)
    assert cn.get_status() == 0


def test_absorbing_step_residual_at_2e24(gpu):
    """At the bench's 2^24 rows: the step's output satisfies T psi_out = (1 - i tau H) psi_in
    (T and the right side built in the test from their definitions with torch ops) to a
    relative residual of 1e-12, a property that holds at any size."""
    torch, cn = gpu
    n, dx, dt = 1 << 24, 0.01, 0.02
    log("absorbing residual", n)
    g = np.random.default_rng(1010)
    V = torch.from_numpy(g.uniform(-1.0, 0.0, n)).cuda()
    W = torch.from_numpy(workloads.absorber(n)).cuda()
    p = torch.from_numpy(workloads.complex_normal(g, n)).cuda()
    out = cn.step(p, V, dx, dt, W=W)
    tau, kap = dt / 2, dt / (4 * dx * dx)
    diag = 1.0 / dx**2 + V
    a = torch.complex(1.0 + tau * W, tau * diag)
    ex = torch.complex(1.0 - tau * W, -tau * diag)

    def nb(x):
        s = torch.zeros_like(x)
        s[1:] += x[:-1]
        s[:-1] += x[1:]
        return s

    lhs = a * out - 1j * kap * nb(out)
    rhs = ex * p + 1j * kap * nb(p)
    res = float(torch.linalg.vector_norm(lhs - rhs) / torch.linalg.vector_norm(rhs))
    assert res <= 1e-12
    assert cn.get_status() == 0
