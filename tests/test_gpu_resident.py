"""GPU parity of the resident propagation (cn_propagate_resident: every step of one system in one
launch, the tiles kept in registers, the reduced system solved by the last workgroup to arrive
at each step) against the CPU oracle stepping one step at a time, and against cn_propagate.

Tolerance: relative L2 <= 1e-11 (FP64 on both sides; rounding only).  Cases: the plain 1D
workload's 200 steps, ragged sizes from one row to 2^20 rows with a field (every tile
configuration: 512, 1024 and 2048 rows), the absorbing workload and absorbing ramps with a
field (the potential V - iW), checkpoints against the oracle's states and the autograd forward
in one launch, a captured graph replayed against the eager result,
the layouts and operators it refuses, and a wait that gives up (forced from the host with a
poll bound of zero), after which the next launch is correct again.
"""
import ctypes
import os

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


def test_resident_plain_1d_200_steps(gpu, oracle_mod):
    """The plain 1D workload (65536 rows, soft-core V, Gaussian packet): 200 steps in one
    launch against the oracle's 200 steps."""
    torch, cn = gpu
    w = workloads.plain_1d()
    log("resident plain_1d", w["n"], w["steps"])
    ref = oracle_mod.cn_propagate(w["psi0"], w["V"], w["dx"], w["dt"], w["steps"])
    tV, tpsi = to_dev(torch, w["V"], w["psi0"])
    cn.propagate_resident(tpsi, tV, w["dx"], w["dt"], w["steps"])
    out = tpsi.cpu().numpy()
    assert rel(out, ref) <= TOL
    assert abs(np.sum(np.abs(out) ** 2) - np.sum(np.abs(w["psi0"]) ** 2)) <= 1e-12 * np.sum(
        np.abs(w["psi0"]) ** 2)
    assert cn.get_status() == 0


@pytest.mark.parametrize("n,part", [(1, 0), (2, 0), (37, 0), (512, 0), (513, 0), (4096, 0),
                                    (65_553, 0), (100_003, 0), (300_007, 0), (1 << 20, 0),
                                    (60_001, 512), (60_001, 1024), (60_001, 2048)])
def test_resident_field_against_oracle(gpu, oracle_mod, n, part):
    """With x E_k in the potential: 7 steps against the oracle's single steps, over ragged
    sizes and each tile configuration (the automatic choice takes the smallest tile whose count
    fits one workgroup's reduced solve)."""
    torch, cn = gpu
    dx, dt, steps = 0.05, 0.01, 7
    log("resident field", n, part)
    inp = workloads.random_cn(n, 41 + n % 89, dx, dt)
    xg = workloads.grid_1d(n, dx)
    E = np.random.default_rng(n % 1000 + part).normal(0.0, 0.05, steps)
    ref = inp["psi"]
    for k in range(steps):
        ref = oracle_mod.cn_step(ref, inp["V"], dx, dt, xg, E[k])
    tV, tpsi, txg = to_dev(torch, inp["V"], inp["psi"], xg)
    L = cn.Layout.contiguous(n, 1, partition=part)
    cn.propagate_resident(tpsi, tV, dx, dt, steps, E=E, xgrid=txg, layout=L)
    assert rel(tpsi.cpu().numpy(), ref) <= TOL
    assert cn.get_status() == 0


def test_resident_absorbing_workload(gpu, oracle_mod):
    """The absorbing workload (packet moving into the ramp at the right wall): 200 steps in one
    launch against the oracle's steps with the potential V - iW, the norm falling."""
    torch, cn = gpu
    w = workloads.absorbing_1d()
    log("resident absorbing", w["n"], w["steps"])
    ref = oracle_mod.cn_propagate(w["psi0"], w["V"], w["dx"], w["dt"], w["steps"], W=w["W"])
    tV, tpsi, tW = to_dev(torch, w["V"], w["psi0"], w["W"])
    cn.propagate_resident(tpsi, tV, w["dx"], w["dt"], w["steps"], W=tW)
    out = tpsi.cpu().numpy()
    assert rel(out, ref) <= TOL
    assert np.sum(np.abs(out) ** 2) < 0.5 * np.sum(np.abs(w["psi0"]) ** 2)
    assert cn.get_status() == 0


@pytest.mark.parametrize("n", [37, 100_003, 300_007])
def test_resident_absorbing_with_field(gpu, oracle_mod, n):
    """An absorbing ramp and x E_k together: 6 steps against the oracle (tiles of 512, 1024
    and 2048 rows)."""
    torch, cn = gpu
    dx, dt, steps = 0.05, 0.01, 6
    inp = workloads.random_cn(n, 23 + n % 61, dx, dt)
    W = workloads.absorber(n, 0.2, 3.0)
    xg = workloads.grid_1d(n, dx)
    E = np.random.default_rng(n % 777).normal(0.0, 0.05, steps)
    ref = inp["psi"]
    for k in range(steps):
        ref = oracle_mod.cn_step(ref, inp["V"], dx, dt, xg, E[k], W=W)
    tV, tpsi, tW, txg = to_dev(torch, inp["V"], inp["psi"], W, xg)
    cn.propagate_resident(tpsi, tV, dx, dt, steps, E=E, xgrid=txg, W=tW)
    assert rel(tpsi.cpu().numpy(), ref) <= TOL
    assert cn.get_status() == 0


@pytest.mark.parametrize("n,steps,K", [(65_536, 30, 7), (300_007, 12, 4), (1 << 20, 9, 3)])
def test_resident_checkpoints(gpu, oracle_mod, n, steps, K):
    """Checkpoints every K steps with a field: each against the oracle's state before that
    step, and equal to those of cn_propagate (the chained passes) to rounding."""
    torch, cn = gpu
    dx, dt = 0.05, 0.01
    log("resident checkpoints", n, steps, K)
    inp = workloads.random_cn(n, 7 + n % 31, dx, dt)
    xg = workloads.grid_1d(n, dx)
    E = np.random.default_rng(n % 101).normal(0.0, 0.05, steps)
    nck = (steps + K - 1) // K
    tV, txg = to_dev(torch, inp["V"], xg)
    a, b = to_dev(torch, inp["psi"], inp["psi"])
    ca = torch.empty(nck * n, dtype=torch.complex128, device="cuda")
    cb = torch.empty_like(ca)
    cn.propagate_resident(a, tV, dx, dt, steps, E=E, xgrid=txg, ckpt=ca, K=K)
    cn.propagate(b, tV, dx, dt, steps, E=E, xgrid=txg, ckpt=cb, K=K)
    ck = ca.cpu().numpy().reshape(nck, n)
    ref = inp["psi"]
    for k in range(steps):
        if k % K == 0:
            assert rel(ck[k // K], ref) <= TOL, k
        ref = oracle_mod.cn_step(ref, inp["V"], dx, dt, xg, E[k])
    assert rel(a.cpu().numpy(), ref) <= TOL
    assert rel(ca.cpu().numpy(), cb.cpu().numpy()) <= 1e-12
    assert cn.get_status() == 0


def test_autograd_resident_forward(gpu):
    """autograd.cn_propagate(resident=True): the forward in one launch with its checkpoints
    gives the state and the gradients of the chained form."""
    torch, cn = gpu
    from paper_2205_00856_amd import autograd as ag

    n, steps, dx, dt = 70_001, 25, 0.05, 0.01
    g = np.random.default_rng(18)
    x = torch.tensor(workloads.grid_1d(n, dx), device="cuda")
    p0 = torch.tensor(workloads.complex_normal(g, n), device="cuda")
    phi = torch.tensor(workloads.complex_normal(g, n), device="cuda")
    V0 = g.uniform(-1.0, 0.0, n)
    E0 = g.normal(0.0, 0.05, steps)
    res = []
    for resident in (False, True):
        V = torch.tensor(V0, device="cuda", requires_grad=True)
        E = torch.tensor(E0, device="cuda", requires_grad=True)
        out = ag.cn_propagate(p0, V, E, dx, dt, xgrid=x, K=6, resident=resident)
        loss = torch.abs((torch.conj(phi) * out).sum() * dx) ** 2
        loss.backward()
        res.append((out.detach().cpu().numpy(), V.grad.cpu().numpy(), E.grad.cpu().numpy()))
    for a, b in zip(res[1], res[0]):
        assert rel(a, b) <= 1e-11


def test_resident_matches_chained_propagation(gpu):
    """The same 60 steps through cn_propagate (fused passes) and in one launch."""
    torch, cn = gpu
    n, dx, dt, steps = 200_003, 0.1, 0.02, 60
    inp = workloads.random_cn(n, 5, dx, dt)
    xg = workloads.grid_1d(n, dx)
    E = np.random.default_rng(9).normal(0.0, 0.05, steps)
    tV, txg = to_dev(torch, inp["V"], xg)
    a, b = to_dev(torch, inp["psi"], inp["psi"])
    cn.propagate(a, tV, dx, dt, steps, E=E, xgrid=txg)
    cn.propagate_resident(b, tV, dx, dt, steps, E=E, xgrid=txg)
    assert rel(b.cpu().numpy(), a.cpu().numpy()) <= 1e-12


def test_resident_graph_replays(gpu):
    """Captured without a field (the buffers sized by one call outside capture), replayed three
    times with eager work and synchronisations between; every replay equals 40 eager steps."""
    torch, cn = gpu
    n, dx, dt, steps = 65_536, 0.1, 0.02, 40
    w = workloads.plain_1d(n=n)
    tV, p0 = to_dev(torch, w["V"], w["psi0"])
    want = p0.clone()
    cn.propagate_resident(want, tV, dx, dt, steps)
    torch.cuda.synchronize()
    psi = p0.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        cn.propagate_resident(psi, tV, dx, dt, 1)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cn.propagate_resident(psi, tV, dx, dt, steps)
    for rep in range(3):
        psi.copy_(p0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert rel(psi.cpu().numpy(), want.cpu().numpy()) <= 1e-14, rep
        _ = (psi * 2).sum().item()  # eager work between replays
    assert cn.get_status() == 0


def test_resident_capture_after_reserve(gpu):
    """On a fresh handle, cn_reserve of the layout sizes the resident buffer, so the first call
    can be a captured one; the replays equal eager steps."""
    torch, cn = gpu
    from paper_2205_00856_amd import _lib
    from paper_2205_00856_amd.api import _operator

    lib = _lib.lib()
    n, dx, dt, steps = 100_003, 0.1, 0.02, 12
    inp = workloads.random_cn(n, 29, dx, dt)
    tV, p0 = to_dev(torch, inp["V"], inp["psi"])
    want = p0.clone()
    cn.propagate_resident(want, tV, dx, dt, steps)
    torch.cuda.synchronize()
    h = ctypes.c_void_p()
    assert lib.cn_create(ctypes.byref(h), 0) == _lib.CN_OK
    try:
        Lc = cn.Layout.contiguous(n, 1).c()
        op = _operator(tV, dx, dt)
        assert lib.cn_reserve(h, ctypes.byref(Lc)) == _lib.CN_OK
        psi = p0.clone()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            st = lib.cn_propagate_resident(h, ctypes.byref(Lc), ctypes.byref(op), steps, None,
                                           ctypes.c_void_p(psi.data_ptr()), None, 1,
                                           ctypes.c_void_p(side.cuda_stream))
        assert st == _lib.CN_OK
        for _ in range(2):
            psi.copy_(p0)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert rel(psi.cpu().numpy(), want.cpu().numpy()) <= 1e-14
        assert lib.cn_get_status(h, None) == _lib.CN_OK
    finally:
        torch.cuda.synchronize()
        lib.cn_destroy(h)


def test_resident_refusals(gpu):
    torch, cn = gpu
    from paper_2205_00856_amd import _lib
    from paper_2205_00856_amd.api import _operator

    lib = _lib.lib()
    n, dx, dt = 4096, 0.1, 0.02
    inp = workloads.random_cn(n, 3, dx, dt)
    tV, tpsi = to_dev(torch, inp["V"], inp["psi"])
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    h = cn.handle(0).ptr

    def call(L, op, steps=3, E=None):
        Lc = L.c()
        return lib.cn_propagate_resident(h, ctypes.byref(Lc), ctypes.byref(op), steps, E,
                                         ctypes.c_void_p(tpsi.data_ptr()), None, 1, s)

    op = _operator(tV, dx, dt)
    U = _lib.CN_ERR_UNSUPPORTED
    assert call(cn.Layout.contiguous(n // 2, 2), op) == U  # a batch
    assert call(cn.Layout.contiguous(n, 1, partition=4096), op) == U  # no such tile
    assert call(cn.Layout.contiguous(n, 1, rows_per_thread=4), op) == U
    assert call(cn.Layout.contiguous(n, 1, levels=1), op) == U
    assert call(cn.Layout.contiguous(1 << 22, 1), op) == U  # more tiles than one solve takes
    tdx = torch.full((1,), dx, dtype=torch.float64, device="cuda")
    assert call(cn.Layout.contiguous(n, 1), _operator(tV, 0.0, dt, dx_per_system=tdx)) == U
    assert call(cn.Layout.contiguous(n, 1), op, steps=-1) == _lib.CN_ERR_INVALID_ARG
    before = tpsi.clone()
    assert call(cn.Layout.contiguous(n, 1), op, steps=0) == _lib.CN_OK  # nothing to do
    torch.cuda.synchronize()
    assert torch.equal(before, tpsi)


def test_resident_wait_bound_reported_then_recovers(gpu, oracle_mod):
    """A poll bound of zero (forced from the host) makes every workgroup that has to wait give
    up at once: each kernel still exits, cn_get_status reports CN_ERR_WAIT_TIMEOUT, and the next
    launch with the normal bound is correct (the hand-over words were reset on the way out)."""
    torch, cn = gpu
    from paper_2205_00856_amd import _lib

    n, dx, dt, steps = 100_003, 0.1, 0.02, 5
    inp = workloads.random_cn(n, 17, dx, dt)
    tV, tpsi = to_dev(torch, inp["V"], inp["psi"])
    os.environ["CN_RESIDENT_SPIN"] = "0"
    try:
        cn.propagate_resident(tpsi, tV, dx, dt, steps)
        torch.cuda.synchronize()
    finally:
        del os.environ["CN_RESIDENT_SPIN"]
    with pytest.raises(_lib.CnError) as e:
        cn.get_status()
    assert e.value.status == _lib.CN_ERR_WAIT_TIMEOUT
    assert cn.get_status() == 0  # cleared
    ref = oracle_mod.cn_propagate(inp["psi"], inp["V"], dx, dt, steps)
    (tpsi,) = to_dev(torch, inp["psi"])
    cn.propagate_resident(tpsi, tV, dx, dt, steps)
    assert rel(tpsi.cpu().numpy(), ref) <= TOL
    assert cn.get_status() == 0
