"""GPU reverse mode: CNSolve and CNPropagate against the oracle, dense autograd and finite
differences.  Reference gradients are computed on the CPU in complex128."""
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
    from paper_2205_00856_amd import autograd as ag

    cn.handle(0)
    return torch, cn, ag


def rel(x, y):
    return float(np.linalg.norm(np.asarray(x) - np.asarray(y)) / np.linalg.norm(np.asarray(y)))


def test_cnsolve_matches_dense_autograd(gpu):
    torch, cn, ag = gpu
    n = 48
    a, b, c, d = workloads.random_system(n, 5, "herm")
    w = np.random.default_rng(1).standard_normal(n)
    # reference: dense solve on the CPU
    ta, tb, tc, td = (torch.tensor(v, requires_grad=True) for v in (a, b, c, d))
    T = torch.diag(ta) + torch.diag(tb[1:], -1) + torch.diag(tc[:-1], 1)
    x = torch.linalg.solve(T, td)
    (torch.abs(x) ** 2 * torch.tensor(w)).sum().backward()
    # GPU
    ga, gb, gc, gd = (torch.tensor(v, device="cuda", requires_grad=True) for v in (a, b, c, d))
    xg = ag.cn_solve(ga, gb, gc, gd)
    (torch.abs(xg) ** 2 * torch.tensor(w, device="cuda")).sum().backward()
    assert rel(xg.detach().cpu(), x.detach()) <= 1e-12
    assert rel(gd.grad.cpu(), td.grad) <= 1e-11
    assert rel(ga.grad.cpu(), ta.grad) <= 1e-11
    assert rel(gb.grad.cpu()[1:], tb.grad[1:]) <= 1e-11
    assert rel(gc.grad.cpu()[:-1], tc.grad[:-1]) <= 1e-11


def test_cnsolve_gradcheck(gpu):
    torch, cn, ag = gpu
    n = 9
    a, b, c, d = workloads.random_system(n, 6, "dd")
    args = [torch.tensor(v, device="cuda", requires_grad=True) for v in (a, b, c, d)]
    b_mask = torch.ones(n, dtype=torch.complex128, device="cuda")
    b_mask[0] = 0
    c_mask = torch.ones(n, dtype=torch.complex128, device="cuda")
    c_mask[-1] = 0

    def f(a_, b_, c_, d_):  # the ignored b[0], c[n-1] are masked so finite differences agree
        return ag.cn_solve(a_, b_ * b_mask, c_ * c_mask, d_)

    assert torch.autograd.gradcheck(f, args, eps=1e-6, atol=1e-8, rtol=1e-6)


@pytest.mark.parametrize("n,steps,K", [(6000, 45, 7), (1 << 20, 5, 2)])
def test_cnpropagate_matches_oracle_reverse_mode(gpu, oracle_mod, n, steps, K):
    torch, cn, ag = gpu
    dx, dt = 0.05, 0.01
    x = workloads.grid_1d(n, dx)
    V = workloads.softcore(x)
    E = np.random.default_rng(2).normal(0, 0.05, steps)
    psi0 = workloads.gaussian(x, 0.0, 5.0, 1.0, dx)
    phi = workloads.gaussian(x, 20.0, 5.0, 1.0, dx)
    psiT = oracle_mod.cn_propagate(psi0, V, dx, dt, steps, x, E)
    G_T = 2 * (np.sum(np.conj(phi) * psiT) * dx) * phi * dx
    g0, dV, dE = oracle_mod.cn_propagate_grad(psi0, V, dx, dt, steps, G_T, x, E)
    tpsi = torch.tensor(psi0, device="cuda", requires_grad=True)
    tV = torch.tensor(V, device="cuda", requires_grad=True)
    tE = torch.tensor(E, device="cuda", requires_grad=True)
    tx = torch.tensor(x, device="cuda")
    out = ag.cn_propagate(tpsi, tV, tE, dx, dt, xgrid=tx, K=K)
    assert rel(out.detach().cpu().numpy(), psiT) <= 1e-11
    ov = (torch.conj(torch.tensor(phi, device="cuda")) * out).sum() * dx
    (torch.abs(ov) ** 2).backward()
    assert rel(tV.grad.cpu().numpy(), dV) <= 1e-10
    assert rel(tE.grad.cpu().numpy(), dE) <= 1e-10
    assert rel(tpsi.grad.cpu().numpy(), g0) <= 1e-10


def test_cnpropagate_finite_differences(gpu):
    """Gradients of |<phi|psi_T>|^2 w.r.t. V_j and E_k against central differences of the
    GPU forward (itself parity-checked against the oracle), 16 coordinates."""
    torch, cn, ag = gpu
    w = workloads.differentiated(n=1 << 14, steps=120, ckpt=25, seed=1004)
    dx, dt = w["dx"], w["dt"]
    tV = torch.tensor(w["V"], device="cuda", requires_grad=True)
    tE = torch.tensor(w["E"], device="cuda", requires_grad=True)
    tx = torch.tensor(w["x"], device="cuda")
    p0 = torch.tensor(w["psi0"], device="cuda")
    phi = torch.tensor(w["phi"], device="cuda")

    def loss(Vt, Et):
        out = ag.cn_propagate(p0, Vt, Et, dx, dt, xgrid=tx, K=w["ckpt"])
        return torch.abs((torch.conj(phi) * out).sum() * dx) ** 2

    L = loss(tV, tE)
    L.backward()
    gV = tV.grad.cpu().numpy()
    gE = tE.grad.cpu().numpy()
    rng = np.random.default_rng(7)
    dens = np.abs(w["psi0"]) ** 2
    js = rng.choice(np.nonzero(dens > 1e-6 * dens.max())[0], 8, replace=False)
    ks = rng.choice(w["steps"], 8, replace=False)
    h = 1e-4
    num, ana = [], []
    with torch.no_grad():
        for j in js:
            Vp = tV.detach().clone()
            Vm = tV.detach().clone()
            Vp[j] += h
            Vm[j] -= h
            num.append(float((loss(Vp, tE.detach()) - loss(Vm, tE.detach())) / (2 * h)))
            ana.append(gV[j])
        for k in ks:
            Ep = tE.detach().clone()
            Em = tE.detach().clone()
            Ep[k] += h
            Em[k] -= h
            num.append(float((loss(tV.detach(), Ep) - loss(tV.detach(), Em)) / (2 * h)))
            ana.append(gE[k])
    assert rel(ana, num) <= 1e-6
