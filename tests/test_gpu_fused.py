"""GPU parity of cn_propagate over two-pass plans, whose steps run as one fused pass each (the
second pass of step k with the first pass of step k+1; the reduced system adds the joint rows'
deferred neighbour terms), against the CPU oracle stepping one step at a time.

Tolerance: relative L2 <= 1e-11 (FP64 on both sides; rounding only).  Cases: one long system
with a field and checkpoints (row tiles of 4 and 8 rows per lane, second passes alternating
direction above 2^21 rows), a uniform batch with a dx per system, an uneven batch mixing
whole-system tiles and two-pass systems, a reduced system that is itself two-pass, 1 and 2
steps, and a captured graph replayed against the eager result.
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


@pytest.mark.parametrize("n", [200_003, 1_048_579, 2_100_003])
def test_propagate_long_system_field_checkpoints(gpu, oracle_mod, n):
    torch, cn = gpu
    log("fused propagate", n)
    dx, dt, steps, K = 0.05, 0.01, 7, 3
    inp = workloads.random_cn(n, 71 + n % 97, dx, dt)
    xg = workloads.grid_1d(n, dx)
    E = np.random.default_rng(n % 1000).normal(0.0, 0.05, steps)
    tV, tpsi, txg = to_dev(torch, inp["V"], inp["psi"], xg)
    L = cn.Layout.contiguous(n, 1)
    ckpt = torch.empty(((steps + K - 1) // K) * n, dtype=torch.complex128, device="cuda")
    cn.propagate(tpsi, tV, dx, dt, steps, E=E, xgrid=txg, ckpt=ckpt, K=K, layout=L)
    ref = inp["psi"]
    states = [ref]
    for k in range(steps):
        ref = oracle_mod.cn_step(ref, inp["V"], dx, dt, xg, E[k])
        states.append(ref)
    assert rel(tpsi.cpu().numpy(), states[steps]) <= TOL
    ck = ckpt.cpu().numpy().reshape(-1, n)
    for j in range(ck.shape[0]):
        assert rel(ck[j], states[j * K]) <= TOL
    assert cn.get_status() == 0


def test_propagate_uniform_batch_dx_per_system(gpu, oracle_mod):
    torch, cn = gpu
    n, batch, dt, steps = 70_001, 3, 0.02, 5
    g = np.random.default_rng(12)
    V = g.uniform(-2.0, 0.0, n * batch)
    psi = workloads.complex_normal(g, n * batch)
    dxs = np.array([0.05, 0.1, 0.17])
    tV, tpsi, tdx = to_dev(torch, V, psi, dxs)
    cn.propagate(tpsi, tV, 1.0, dt, steps, dx_per_system=tdx, layout=cn.Layout.contiguous(n, batch))
    out = tpsi.cpu().numpy()
    for s in range(batch):
        ref = oracle_mod.cn_propagate(psi[s * n:(s + 1) * n], V[s * n:(s + 1) * n], dxs[s], dt,
                                      steps)
        assert rel(out[s * n:(s + 1) * n], ref) <= TOL


def test_propagate_uneven_mixed(gpu, oracle_mod):
    torch, cn = gpu
    lengths = np.array([1, 5, 300, 4096, 4097, 9000, 20_000, 65_543, 2, 100_000, 2048, 33_333])
    offs = np.zeros(lengths.size + 1, np.int64)
    np.cumsum(lengths, out=offs[1:])
    g = np.random.default_rng(13)
    V = g.uniform(-2.0, 0.0, offs[-1])
    psi = workloads.complex_normal(g, offs[-1])
    dxs = g.uniform(0.05, 0.2, lengths.size)
    dt, steps = 0.02, 4
    tV, tpsi, tdx = to_dev(torch, V, psi, dxs)
    L = cn.Layout.uneven(offs)
    log("uneven fused plan:", cn.describe_plan(L, True))
    cn.propagate(tpsi, tV, 1.0, dt, steps, dx_per_system=tdx, layout=L)
    ref = psi
    for _ in range(steps):
        ref = oracle_mod.cn_step_batched(offs, ref, V, dxs, dt)
    assert rel(tpsi.cpu().numpy(), ref) <= TOL


def test_propagate_two_pass_reduced_system(gpu, oracle_mod):
    """2^24 + 5 rows: 8193 first-level tiles, whose reduced system is solved in two passes
    as well (the deferred terms enter both of its passes)."""
    torch, cn = gpu
    n, dx, dt, steps = (1 << 24) + 5, 0.1, 0.02, 3
    inp = workloads.random_cn(n, 5, dx, dt)
    tV, tpsi = to_dev(torch, inp["V"], inp["psi"])
    L = cn.Layout.contiguous(n, 1)
    log("two-level plan:", cn.describe_plan(L, True))
    cn.propagate(tpsi, tV, dx, dt, steps, layout=L)
    ref = oracle_mod.cn_propagate(inp["psi"], inp["V"], dx, dt, steps)
    assert rel(tpsi.cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("steps", [1, 2])
def test_propagate_few_steps(gpu, oracle_mod, steps):
    torch, cn = gpu
    n, dx, dt = 100_003, 0.1, 0.02
    inp = workloads.random_cn(n, 17, dx, dt)
    tV, tpsi = to_dev(torch, inp["V"], inp["psi"])
    cn.propagate(tpsi, tV, dx, dt, steps)
    ref = oracle_mod.cn_propagate(inp["psi"], inp["V"], dx, dt, steps)
    assert rel(tpsi.cpu().numpy(), ref) <= TOL


def test_propagate_fused_graph_replays(gpu):
    """The fused sequence captured as a graph, replayed with eager work between the replays,
    gives the eager result bit for bit."""
    torch, cn = gpu
    n, dx, dt, steps = 300_001, 0.1, 0.02, 6
    inp = workloads.random_cn(n, 23, dx, dt)
    tV, p0 = to_dev(torch, inp["V"], inp["psi"])
    L = cn.Layout.contiguous(n, 1)
    cn.reserve(L)
    eager = p0.clone()
    cn.propagate(eager, tV, dx, dt, steps, layout=L)
    psi = p0.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        cn.propagate(psi, tV, dx, dt, steps, layout=L)
    for _ in range(3):
        psi.copy_(p0)
        graph.replay()
        torch.cuda.synchronize()
        junk = p0.clone()
        cn.propagate(junk, tV, dx, dt, 2, layout=L)
        torch.cuda.synchronize()
        assert torch.equal(psi, eager)


# ------------------------------------------------------------------ reverse mode on g
def _reverse_case(torch, cn, oracle_mod, n, batch, steps, K, interleaved=False, seed=0):
    """cn_propagate with checkpoints, then cn_propagate_adjoint, against the oracle's reverse
    mode per system (dE summed over the systems, as the library sums over all rows)."""
    dx, dt = 0.05, 0.01
    g = np.random.default_rng(seed)
    x1 = workloads.grid_1d(n, dx)
    V = g.uniform(-1.0, 0.0, (batch, n))
    P0 = workloads.complex_normal(g, (batch, n))
    GT = workloads.complex_normal(g, (batch, n))
    E = g.normal(0.0, 0.05, steps)
    X = np.tile(x1, (batch, 1))
    if interleaved:
        L = cn.Layout.interleaved(n, batch)
        lay = lambda a: np.ascontiguousarray(a.T).ravel()  # noqa: E731
    else:
        L = cn.Layout.contiguous(n, batch)
        lay = lambda a: np.ascontiguousarray(a).ravel()  # noqa: E731
    tV, tx, tp, tg = to_dev(torch, lay(V), lay(X), lay(P0), lay(GT))
    nseg = (steps + K - 1) // K
    ckpt = torch.empty(nseg * n * batch, dtype=torch.complex128, device="cuda")
    cn.propagate(tp, tV, dx, dt, steps, E=E, xgrid=tx, ckpt=ckpt, K=K, layout=L)
    dV = torch.zeros(n * batch, dtype=torch.float64, device="cuda")
    dE = torch.zeros(steps, dtype=torch.float64, device="cuda")
    cn.propagate_adjoint(ckpt, tg, tV, dx, dt, steps, K, E=E, xgrid=tx, dV=dV, dE=dE, layout=L)
    unlay = (lambda t: t.cpu().numpy().reshape(n, batch).T) if interleaved else \
        (lambda t: t.cpu().numpy().reshape(batch, n))
    g0, gV = unlay(tg), unlay(dV)
    dE_ref = np.zeros(steps)
    for s in range(batch):
        r0, rV, rE = oracle_mod.cn_propagate_grad(P0[s], V[s], dx, dt, steps, GT[s], x1, E)
        assert rel(g0[s], r0) <= 1e-10, s
        assert rel(gV[s], rV) <= 1e-10, s
        dE_ref += rE
    assert rel(dE.cpu().numpy(), dE_ref) <= 1e-10
    assert cn.get_status() == 0


@pytest.mark.parametrize("n,steps,K", [(5000, 3, 10), (5000, 4, 1), (5000, 1, 3), (3000, 5, 2)])
def test_reverse_mode_segments(gpu, oracle_mod, n, steps, K):
    """One segment (serial chain, recompute on the second workspace), one step per segment
    (the chain crosses a segment at every step), a single step, and single-tile systems
    (no fusable group: steps one at a time)."""
    torch, cn = gpu
    log("reverse", n, steps, K)
    _reverse_case(torch, cn, oracle_mod, n, 1, steps, K, seed=n + steps + K)


def test_reverse_mode_interleaved_batch(gpu, oracle_mod):
    """64 interleaved systems: the column kernels form lambda = (g_k + g_{k+1}) / 2 at their
    store; segments overlapped on the second stream."""
    torch, cn = gpu
    _reverse_case(torch, cn, oracle_mod, 300, 64, 5, 2, interleaved=True, seed=3)


def test_reverse_mode_uniform_batch_two_pass(gpu, oracle_mod):
    """3 contiguous systems of 20 000 rows: the fused chain over a batch, 7 steps, K = 3."""
    torch, cn = gpu
    _reverse_case(torch, cn, oracle_mod, 20_000, 3, 7, 3, seed=11)


def test_reverse_mode_captured_after_reserve_only(gpu):
    """A layout no call has used yet: after cn_reserve alone, the reverse mode (dV, no dE) is
    captured and replayed; every replay equals an eager call bit for bit (both run the fused
    chain, the capture with its segments one after the other)."""
    torch, cn = gpu
    n, dx, dt, steps, K = 40_003, 0.05, 0.01, 9, 4
    g = np.random.default_rng(31)
    V = g.uniform(-1.0, 0.0, n)
    tV, tp, tg = to_dev(torch, V, workloads.complex_normal(g, n), workloads.complex_normal(g, n))
    L = cn.Layout.contiguous(n, 1)
    cn.reserve(L)
    ckpt = torch.empty(((steps + K - 1) // K) * n, dtype=torch.complex128, device="cuda")
    seg = torch.empty((K + 1) * n, dtype=torch.complex128, device="cuda")
    gc = torch.empty_like(tg)
    dVc = torch.zeros(n, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        cn.propagate(tp, tV, dx, dt, steps, ckpt=ckpt, K=K, layout=L)
        cn.propagate_adjoint(ckpt, gc, tV, dx, dt, steps, K, dV=dVc, seg=seg, layout=L)
    p0 = tp.clone()
    for _ in range(3):
        tp.copy_(p0)
        gc.copy_(tg)
        dVc.zero_()
        graph.replay()
        torch.cuda.synchronize()
        pe = p0.clone()
        cn.propagate(pe, tV, dx, dt, steps, ckpt=ckpt, K=K, layout=L)
        ge = tg.clone()
        dVe = torch.zeros(n, dtype=torch.float64, device="cuda")
        cn.propagate_adjoint(ckpt, ge, tV, dx, dt, steps, K, dV=dVe, seg=seg, layout=L)
        torch.cuda.synchronize()
        assert torch.equal(gc, ge) and torch.equal(dVc, dVe)


# ------------------------------------------------ reduced system solved inside the fused pass
# One system in K tiles whose K joints fill more than half of a whole-system tile of 2 rows per
# lane of the pass's workgroup (64 W < K <= 128 W): the pass's last workgroup solves the reduced
# system, so a step is one launch.  The automatic 2^20 plan (512 tiles of 2048 rows, W = 4, the
# cap), 100 tiles of 128 rows (W = 1), 196 tiles of 512 (W = 2, a last tile of 163 rows), 301
# tiles of 2048 (a last tile of one row); with a field and checkpoints.
@pytest.mark.parametrize("n,T,M", [(1 << 20, 0, 0), (12_800, 128, 2), (100_003, 512, 4),
                                   (614_401, 2048, 8)])
def test_propagate_reduced_system_in_pass(gpu, oracle_mod, n, T, M):
    torch, cn = gpu
    log("reduced system in the pass", n, T, M)
    dx, dt, steps, K = 0.05, 0.01, 12, 5
    inp = workloads.random_cn(n, 5 + n % 89, dx, dt)
    xg = workloads.grid_1d(n, dx)
    E = np.random.default_rng(n % 777).normal(0.0, 0.05, steps)
    L = cn.Layout.contiguous(n, 1, partition=T, rows_per_thread=M)
    plan = cn.describe_plan(L, cn_mode=True)
    log(plan)
    assert "reduced system solved in the pass" in plan
    tV, tpsi, txg = to_dev(torch, inp["V"], inp["psi"], xg)
    ckpt = torch.empty(((steps + K - 1) // K) * n, dtype=torch.complex128, device="cuda")
    cn.propagate(tpsi, tV, dx, dt, steps, E=E, xgrid=txg, ckpt=ckpt, K=K, layout=L)
    ref = inp["psi"]
    states = [ref]
    for k in range(steps):
        ref = oracle_mod.cn_step(ref, inp["V"], dx, dt, xg, E[k])
        states.append(ref)
    assert rel(tpsi.cpu().numpy(), states[steps]) <= TOL
    ck = ckpt.cpu().numpy().reshape(-1, n)
    for j in range(ck.shape[0]):
        assert rel(ck[j], states[j * K]) <= TOL
    assert cn.get_status() == 0


def test_reduced_system_in_pass_graph_and_reverse(gpu, oracle_mod):
    """The one-launch steps captured as a graph and replayed with eager work between the
    replays (the done count is back at zero after every pass), and the reverse mode, whose
    recompute runs the same chain on the second workspace and stream beside the recursion."""
    torch, cn = gpu
    n, dx, dt, steps = 100_003, 0.1, 0.02, 9
    L = cn.Layout.contiguous(n, 1, partition=512, rows_per_thread=4)
    assert "reduced system solved in the pass" in cn.describe_plan(L, cn_mode=True)
    inp = workloads.random_cn(n, 29, dx, dt)
    tV, p0 = to_dev(torch, inp["V"], inp["psi"])
    cn.reserve(L)
    eager = p0.clone()
    cn.propagate(eager, tV, dx, dt, steps, layout=L)
    ref = oracle_mod.cn_propagate(inp["psi"], inp["V"], dx, dt, steps)
    assert rel(eager.cpu().numpy(), ref) <= TOL
    psi = p0.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        cn.propagate(psi, tV, dx, dt, steps, layout=L)
    for _ in range(4):
        psi.copy_(p0)
        graph.replay()
        torch.cuda.synchronize()
        junk = p0.clone()
        cn.propagate(junk, tV, dx, dt, 3, layout=L)
        torch.cuda.synchronize()
        assert torch.equal(psi, eager)
    # reverse mode: 4 segments of 5 steps, recomputes overlapped on the second stream
    nst, K = 20, 5
    x1 = workloads.grid_1d(n, dx)
    g = np.random.default_rng(3)
    GT = workloads.complex_normal(g, n)
    E = g.normal(0.0, 0.05, nst)
    tp, tg, tx = to_dev(torch, inp["psi"], GT, x1)
    ckpt = torch.empty((nst // K) * n, dtype=torch.complex128, device="cuda")
    cn.propagate(tp, tV, dx, dt, nst, E=E, xgrid=tx, ckpt=ckpt, K=K, layout=L)
    dV = torch.zeros(n, dtype=torch.float64, device="cuda")
    dE = torch.zeros(nst, dtype=torch.float64, device="cuda")
    cn.propagate_adjoint(ckpt, tg, tV, dx, dt, nst, K, E=E, xgrid=tx, dV=dV, dE=dE, layout=L)
    r0, rV, rE = oracle_mod.cn_propagate_grad(inp["psi"], inp["V"], dx, dt, nst, GT, x1, E)
    assert rel(tg.cpu().numpy(), r0) <= 1e-10
    assert rel(dV.cpu().numpy(), rV) <= 1e-10
    assert rel(dE.cpu().numpy(), rE) <= 1e-10
    assert cn.get_status() == 0


# ------------------------------------------------------ reverse mode without checkpoints
@pytest.mark.parametrize("n,steps,K,T,M", [(100_003, 23, 5, 0, 0), (65536, 40, 7, 512, 4),
                                           (1 << 20, 30, 10, 0, 0), (3000, 6, 4, 0, 0),
                                           (50_000, 9, 20, 0, 0)])
def test_reverse_reconstruction(gpu, oracle_mod, n, steps, K, T, M):
    """cn_propagate_adjoint_reconstruct: no checkpoints; each segment's states are rebuilt
    backwards from the state at its end (psi_T for the last), a CN step with -dt, beside the
    recursion on g.  Against the oracle's reverse mode (which steps forward from psi_0) and the
    checkpointed GPU reverse mode; psi_T is left untouched.  Cases: fused chains in segments of
    5, 7 and 10 steps (the 2^20 one with its reduced system solved in the pass), whole-system
    tiles stepped one at a time, one segment longer than the sequence."""
    torch, cn = gpu
    log("reverse reconstruction", n, steps, K, T, M)
    dx, dt = 0.05, 0.01
    g = np.random.default_rng(n % 1000 + steps)
    x1 = workloads.grid_1d(n, dx)
    V = g.uniform(-1.0, 0.0, n)
    P0 = workloads.complex_normal(g, n)
    GT = workloads.complex_normal(g, n)
    E = g.normal(0.0, 0.05, steps)
    L = cn.Layout.contiguous(n, 1, partition=T, rows_per_thread=M)
    tV, tx, tp, tg = to_dev(torch, V, x1, P0, GT)
    cn.propagate(tp, tV, dx, dt, steps, E=E, xgrid=tx, layout=L)
    psiT = tp.clone()
    dV = torch.zeros(n, dtype=torch.float64, device="cuda")
    dE = torch.zeros(steps, dtype=torch.float64, device="cuda")
    cn.propagate_adjoint_reconstruct(tp, tg, tV, dx, dt, steps, K, E=E, xgrid=tx, dV=dV, dE=dE,
                                     layout=L)
    assert torch.equal(tp, psiT)
    r0, rV, rE = oracle_mod.cn_propagate_grad(P0, V, dx, dt, steps, GT, x1, E)
    assert rel(tg.cpu().numpy(), r0) <= 1e-10
    assert rel(dV.cpu().numpy(), rV) <= 1e-10
    assert rel(dE.cpu().numpy(), rE) <= 1e-10
    # the checkpointed reverse mode on the same forward
    tp2 = to_dev(torch, P0)[0]
    ckpt = torch.empty(((steps + K - 1) // K) * n, dtype=torch.complex128, device="cuda")
    cn.propagate(tp2, tV, dx, dt, steps, E=E, xgrid=tx, ckpt=ckpt, K=K, layout=L)
    g2 = to_dev(torch, GT)[0]
    dV2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    dE2 = torch.zeros(steps, dtype=torch.float64, device="cuda")
    cn.propagate_adjoint(ckpt, g2, tV, dx, dt, steps, K, E=E, xgrid=tx, dV=dV2, dE=dE2,
                         layout=L)
    assert rel(tg.cpu().numpy(), g2.cpu().numpy()) <= 1e-11
    assert rel(dV.cpu().numpy(), dV2.cpu().numpy()) <= 1e-11
    assert cn.get_status() == 0


def test_reverse_reconstruction_refuses_absorbing(gpu):
    """The inverse of a step with an absorbing potential amplifies: refused."""
    torch, cn = gpu
    from paper_2205_00856_amd._lib import CnError

    n = 4096
    tV = torch.zeros(n, dtype=torch.float64, device="cuda")
    W = torch.full((n,), 0.1, dtype=torch.float64, device="cuda")
    p = torch.ones(n, dtype=torch.complex128, device="cuda")
    g = torch.ones(n, dtype=torch.complex128, device="cuda")
    with pytest.raises(CnError):
        cn.propagate_adjoint_reconstruct(p, g, tV, 0.1, 0.01, 4, 2, W=W)


def test_autograd_reconstruct_matches_checkpointed(gpu):
    """autograd.cn_propagate(reconstruct=True) gives the gradients of the checkpointed form."""
    torch, cn = gpu
    from paper_2205_00856_amd import autograd as ag

    n, steps, dx, dt = 20_000, 25, 0.05, 0.01
    g = np.random.default_rng(8)
    x = torch.tensor(workloads.grid_1d(n, dx), device="cuda")
    p0 = torch.tensor(workloads.complex_normal(g, n), device="cuda")
    phi = torch.tensor(workloads.complex_normal(g, n), device="cuda")
    V0 = g.uniform(-1.0, 0.0, n)
    E0 = g.normal(0.0, 0.05, steps)
    grads = []
    for rec in (False, True):
        V = torch.tensor(V0, device="cuda", requires_grad=True)
        E = torch.tensor(E0, device="cuda", requires_grad=True)
        out = ag.cn_propagate(p0, V, E, dx, dt, xgrid=x, K=6, reconstruct=rec)
        loss = torch.abs((torch.conj(phi) * out).sum() * dx) ** 2
        loss.backward()
        grads.append((V.grad.cpu().numpy(), E.grad.cpu().numpy()))
    assert rel(grads[1][0], grads[0][0]) <= 1e-11
    assert rel(grads[1][1], grads[0][1]) <= 1e-11
