"""GPU parity at the benchmark's full sizes, in the launch configurations bench.py times:

* one Lie-split ADI step of the 4096 x 4096 grid (x-sweep over 4096 contiguous lines, y-sweep
  over 4096 interleaved lines, V/2 each), against the oracle's ADI step of the whole grid;
* the 2^28-unknown explicit solve of the seeded workload with the automatic plan, against the
  oracle's Thomas solve of the same arrays, and by its residual (computed on the device with
  plain tensor ops), which bounds the forward error because T's Hermitian part is I;
* one CN step of the whole uneven batch (10^4 systems), system by system against the oracle;
* one 2^22-row matrix with 16 right-hand sides, each against the oracle;
* each workload's full run: the 100 captured ADI steps, the 50 steps of the uneven batch, and
  the differentiated workload's 2000 steps (psi_T and the loss), each against the oracle's run,
  plus that workload's gradients against finite differences on 64 coordinates.

Tolerances: relative L2 <= 1e-11 against the oracle (FP64 on both sides; rounding only);
relative residual <= 1e-13 for the solve (backward-stable elimination of a diagonally dominant
system); gradients within 1e-6 of central differences (relative L2 over the 64 coordinates).
"""
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

    cn.handle(0)
    return torch, cn


def log(*a):
    print(*a, flush=True)


def test_adi_full_grid_one_step(gpu, oracle_mod):
    torch, cn = gpu
    log("ADI 4096^2 one step")
    w = workloads.adi_2d()
    ny, nx = w["psi0"].shape
    ref = oracle_mod.adi_step(w["psi0"], w["V"], w["dx"], w["dy"], w["dt"],
                              oracle_mod.max_threads())
    tV = torch.from_numpy(w["V"].ravel()).cuda()
    p = torch.from_numpy(w["psi0"].ravel()).cuda()
    Lx = cn.Layout.contiguous(nx, ny)
    Ly = cn.Layout.interleaved(ny, nx)
    cn.step(p, tV, w["dx"], w["dt"], v_scale=0.5, out=p, layout=Lx)
    cn.step(p, tV, w["dy"], w["dt"], v_scale=0.5, out=p, layout=Ly)
    out = p.cpu().numpy().reshape(ny, nx)
    err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
    assert err <= 1e-11
    # every line, not only the whole grid: the worst row and column
    rows = np.linalg.norm(out - ref, axis=1) / np.linalg.norm(ref, axis=1)
    cols = np.linalg.norm(out - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert max(rows.max(), cols.max()) <= 1e-11
    assert cn.get_status() == 0


@pytest.mark.timeout(600)
def test_large_system_2e28_against_oracle(gpu, oracle_mod):
    """The 2^28-unknown solve on the seeded workload (V_j ~ U(-1, 0), d complex normal, drawn
    by workloads.large_system), a, b, c assembled on the GPU and solved with the automatic plan,
    against the oracle's assembly and serial Thomas solve of the same arrays."""
    torch, cn = gpu
    log("2^28 solve: drawing the seeded inputs")
    w = workloads.large_system()
    N = w["n"]
    log("2^28 solve: GPU assemble + solve")
    tV = torch.from_numpy(w["V"]).cuda()
    a, b, c = cn.assemble(tV, w["dx"], w["dt"])
    del tV
    d = torch.from_numpy(w["d"]).cuda()
    x = cn.solve(a, b, c, d, layout=cn.Layout.contiguous(N, 1))
    # T's Hermitian part is the identity, so sigma_min(T) >= 1 and |x - x*| <= |T x - d|:
    # the residual relative to |x| bounds the relative forward error rigorously
    r = a * x
    r[1:] += b[1:] * x[:-1]
    r[:-1] += c[:-1] * x[1:]
    r -= d
    rn = float(torch.linalg.vector_norm(r))
    fwd_bound = rn / float(torch.linalg.vector_norm(x))
    resid = rn / float(torch.linalg.vector_norm(d))
    del r, a, b, c, d
    got = x.cpu().numpy()
    del x
    torch.cuda.empty_cache()
    assert cn.get_status() == 0
    assert np.isfinite(got).all()
    assert resid <= 1e-13
    assert fwd_bound <= 1e-11
    log("2^28 solve: oracle assembly + Thomas")
    oa, ob, oc = oracle_mod.cn_coeffs(w["V"], w["dx"], w["dt"])
    ref = oracle_mod.thomas(oa, ob, oc, w["d"])
    del oa, ob, oc
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    log(f"2^28 solve: rel L2 {err:.3e}, forward-error bound {fwd_bound:.3e}")
    assert err <= 1e-11


def test_uneven_batch_full_one_step(gpu, oracle_mod):
    """The full uneven batch (10^4 systems, about 1.18e8 rows) with its automatic plan: one CN
    step against the oracle, checked system by system."""
    torch, cn = gpu
    log("uneven batch full size, one step")
    wl = workloads.uneven_batch()
    offs = wl["offsets"]
    ref = oracle_mod.cn_step_batched(offs, wl["psi0"], wl["V"], wl["dx"], wl["dt"],
                                     oracle_mod.max_threads())
    tV = torch.from_numpy(wl["V"]).cuda()
    tp = torch.from_numpy(wl["psi0"]).cuda()
    tdx = torch.from_numpy(wl["dx"]).cuda()
    out = cn.step(tp, tV, 0.0, wl["dt"], dx_per_system=tdx,
                  layout=cn.Layout.uneven(offs)).cpu().numpy()
    del tV, tp, tdx
    diff = np.abs(out - ref) ** 2
    den = np.abs(ref) ** 2
    num_s = np.add.reduceat(diff, offs[:-1])
    den_s = np.add.reduceat(den, offs[:-1])
    assert np.sqrt(num_s.sum() / den_s.sum()) <= 1e-11
    assert np.sqrt((num_s / den_s).max()) <= 1e-11
    assert cn.get_status() == 0


def test_one_matrix_16_rhs_2e22(gpu, oracle_mod):
    """One 2^22-row matrix with 16 right-hand sides (shared coefficients), every right-hand side
    against the oracle's Thomas solve."""
    torch, cn = gpu
    log("2^22 x 16 shared solve")
    n, k = 1 << 22, 16
    g = torch.Generator(device="cuda")
    g.manual_seed(1006)
    V = torch.rand(n, dtype=torch.float64, device="cuda", generator=g) - 1.0
    a, b, c = cn.assemble(V, 0.01, 0.02)
    d = torch.empty(k * n, dtype=torch.complex128, device="cuda")
    d.real.normal_(generator=g)
    d.imag.normal_(generator=g)
    x = cn.solve(a, b, c, d, layout=cn.Layout.contiguous(n, k, shared_coefficients=True))
    a0, b0, c0 = (t.cpu().numpy() for t in (a, b, c))
    dd = d.cpu().numpy()
    xx = x.cpu().numpy()
    del a, b, c, d, x, V
    torch.cuda.empty_cache()
    for s in range(k):
        ref = oracle_mod.thomas(a0, b0, c0, dd[s * n:(s + 1) * n])
        got = xx[s * n:(s + 1) * n]
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-11, s


@pytest.mark.timeout(600)
def test_adi_full_grid_100_steps_graph(gpu, oracle_mod):
    """The whole ADI workload as bench.py runs it: one step captured as a HIP graph, replayed
    100 times from psi0, against the oracle's 100 ADI steps."""
    torch, cn = gpu
    log("ADI 4096^2, 100 graph replays")
    w = workloads.adi_2d()
    ny, nx = w["psi0"].shape
    tV = torch.from_numpy(w["V"].ravel()).cuda()
    psi = torch.from_numpy(w["psi0"].ravel()).cuda()
    Lx = cn.Layout.contiguous(nx, ny)
    Ly = cn.Layout.interleaved(ny, nx)
    cn.reserve(Lx)
    cn.reserve(Ly)
    p0 = psi.clone()

    def step():
        cn.step(psi, tV, w["dx"], w["dt"], v_scale=0.5, out=psi, layout=Lx)
        cn.step(psi, tV, w["dy"], w["dt"], v_scale=0.5, out=psi, layout=Ly)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    psi.copy_(p0)
    for _ in range(w["steps"]):
        graph.replay()
    torch.cuda.synchronize()
    got = psi.cpu().numpy().reshape(ny, nx)
    del graph, psi, p0, tV
    assert cn.get_status() == 0
    state = w["psi0"]
    nthr = oracle_mod.max_threads()
    for _ in range(w["steps"]):
        state = oracle_mod.adi_step(state, w["V"], w["dx"], w["dy"], w["dt"], nthr)
    err = np.linalg.norm(got - state) / np.linalg.norm(state)
    log(f"ADI 100 steps: rel L2 {err:.3e}")
    assert err <= 1e-11


@pytest.mark.timeout(600)
def test_uneven_batch_50_steps_propagate(gpu, oracle_mod):
    """The whole uneven workload: 50 steps of cn_propagate with the automatic plan (two-pass
    systems fused across steps) against 50 batched oracle steps, system by system."""
    torch, cn = gpu
    log("uneven batch, 50 steps of cn_propagate")
    wl = workloads.uneven_batch()
    offs = wl["offsets"]
    tV = torch.from_numpy(wl["V"]).cuda()
    tp = torch.from_numpy(wl["psi0"]).cuda()
    tdx = torch.from_numpy(wl["dx"]).cuda()
    cn.propagate(tp, tV, 0.0, wl["dt"], wl["steps"], dx_per_system=tdx,
                 layout=cn.Layout.uneven(offs))
    got = tp.cpu().numpy()
    del tV, tp, tdx
    assert cn.get_status() == 0
    ref = wl["psi0"]
    nthr = oracle_mod.max_threads()
    for _ in range(wl["steps"]):
        ref = oracle_mod.cn_step_batched(offs, ref, wl["V"], wl["dx"], wl["dt"], nthr)
    num_s = np.add.reduceat(np.abs(got - ref) ** 2, offs[:-1])
    den_s = np.add.reduceat(np.abs(ref) ** 2, offs[:-1])
    err = np.sqrt(num_s.sum() / den_s.sum())
    worst = np.sqrt((num_s / den_s).max())
    log(f"uneven 50 steps: rel L2 {err:.3e}, worst system {worst:.3e}")
    assert err <= 1e-11
    assert worst <= 1e-11


@pytest.fixture(scope="module")
def differentiated(gpu):
    torch, cn = gpu
    from paper_2205_00856_amd import autograd as ag

    w = workloads.differentiated()
    dev = torch.device("cuda")
    t = dict(V=torch.tensor(w["V"], device=dev), E=torch.tensor(w["E"], device=dev),
             x=torch.tensor(w["x"], device=dev), psi0=torch.tensor(w["psi0"], device=dev),
             phi=torch.tensor(w["phi"], device=dev))

    def forward(Vt, Et):
        return ag.cn_propagate(t["psi0"], Vt, Et, w["dx"], w["dt"], xgrid=t["x"], K=w["ckpt"])

    def loss_of(out):
        return torch.abs((torch.conj(t["phi"]) * out).sum() * w["dx"]) ** 2

    return w, t, forward, loss_of


@pytest.mark.timeout(900)
def test_differentiated_full_length_against_oracle(gpu, oracle_mod, differentiated):
    """The differentiated workload's forward over all 2000 steps (checkpointed every 50, as the
    autograd function runs it): psi_T and the loss |<phi|psi_T>|^2 against the oracle's 2000
    steps."""
    torch, cn = gpu
    w, t, forward, loss_of = differentiated
    log("differentiated: GPU forward, 2000 steps")
    with torch.no_grad():
        out = forward(t["V"], t["E"])
        loss = float(loss_of(out))
    got = out.cpu().numpy()
    assert cn.get_status() == 0
    log("differentiated: oracle, 2000 steps")
    ref = oracle_mod.cn_propagate(w["psi0"], w["V"], w["dx"], w["dt"], w["steps"], w["x"], w["E"])
    ref_loss = abs(np.sum(np.conj(w["phi"]) * ref) * w["dx"]) ** 2
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    lerr = abs(loss - ref_loss) / ref_loss
    log(f"differentiated: psi_T rel L2 {err:.3e}, loss rel {lerr:.3e}")
    assert err <= 1e-11
    assert lerr <= 1e-11


@pytest.mark.timeout(600)
def test_differentiated_full_size_finite_differences(gpu, differentiated):
    """Gradients of the differentiated workload (2^20 rows, 2000 steps, checkpoint 50) w.r.t. 32
    coordinates of V (where psi0 or phi is not negligible) and 32 of E, against central
    differences of the forward with h = 1e-4: relative L2 over the 64 values <= 1e-6."""
    torch, cn = gpu
    w, t, forward, loss_of = differentiated
    log("differentiated: forward + backward")
    tV = t["V"].clone().requires_grad_(True)
    tE = t["E"].clone().requires_grad_(True)
    loss_of(forward(tV, tE)).backward()
    gV = tV.grad.cpu().numpy()
    gE = tE.grad.cpu().numpy()
    rng = np.random.default_rng(2004)
    dens = np.abs(w["psi0"]) ** 2 + np.abs(w["phi"]) ** 2
    js = rng.choice(np.nonzero(dens > 1e-6 * dens.max())[0], 32, replace=False)
    ks = rng.choice(w["steps"], 32, replace=False)
    h = 1e-4
    num, ana = [], []
    log("differentiated: 128 forwards for the finite differences")
    with torch.no_grad():
        for j in js:
            Vp, Vm = t["V"].clone(), t["V"].clone()
            Vp[j] += h
            Vm[j] -= h
            num.append(float(loss_of(forward(Vp, t["E"])) - loss_of(forward(Vm, t["E"]))) / (2 * h))
            ana.append(gV[j])
        for k in ks:
            Ep, Em = t["E"].clone(), t["E"].clone()
            Ep[k] += h
            Em[k] -= h
            num.append(float(loss_of(forward(t["V"], Ep)) - loss_of(forward(t["V"], Em))) / (2 * h))
            ana.append(gE[k])
    num = np.asarray(num)
    ana = np.asarray(ana)
    err = np.linalg.norm(ana - num) / np.linalg.norm(num)
    log(f"differentiated: FD rel L2 over 64 coordinates {err:.3e}")
    assert err <= 1e-6
