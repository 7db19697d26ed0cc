"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

Each test checks the oracle against something other than itself: LAPACK (dense LU and the
banded pivoted solver), exact constructions, the closed-form CN phase on sine modes, unitarity,
time reversal, and a dense restatement of the Hamiltonian.  A dropped term, a wrong sign, a
swapped sub/super diagonal or a wrong index in the oracle fails at least one of them.
"""
import numpy as np
import pytest
import scipy.linalg

import workloads


def dense(a, b, c):
    n = a.shape[0]
    T = np.diag(a).astype(np.complex128)
    if n > 1:
        T += np.diag(b[1:], -1) + np.diag(c[:-1], 1)
    return T


def rel(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


# ------------------------------------------------------------------------- the solve (O3)
@pytest.mark.parametrize("kind", ["dd", "herm"])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 64])
def test_thomas_matches_dense_lu(oracle_mod, kind, n):
    a, b, c, d = workloads.random_system(n, 10 + n, kind)
    x = oracle_mod.thomas(a, b, c, d)
    ref = np.linalg.solve(dense(a, b, c), d)  # LAPACK zgesv, partial pivoting
    assert rel(x, ref) <= 1e-13


def test_thomas_ignores_b0_and_cn(oracle_mod):
    a, b, c, d = workloads.random_system(9, 3, "dd")
    b2, c2 = b.copy(), c.copy()
    b2[0] = 1e300
    c2[-1] = np.nan
    np.testing.assert_array_equal(oracle_mod.thomas(a, b, c, d), oracle_mod.thomas(a, b2, c2, d))


def test_thomas_exact_construction(oracle_mod):
    # Gaussian-integer x and T give an exactly representable d = T x; the solve must return x.
    g = np.random.default_rng(7)
    n = 40
    x = g.integers(-9, 10, n) + 1j * g.integers(-9, 10, n)
    b = g.integers(-3, 4, n) + 1j * g.integers(-3, 4, n)
    c = g.integers(-3, 4, n) + 1j * g.integers(-3, 4, n)
    a = (np.abs(b.real) + np.abs(b.imag) + np.abs(c.real) + np.abs(c.imag) + 2) * (1 + 1j)
    b[0] = 0
    c[-1] = 0
    d = dense(a, b, c) @ x
    assert rel(oracle_mod.thomas(a, b, c, d), x) <= 1e-14


@pytest.mark.parametrize("n", [1000, 200_003])
def test_thomas_matches_lapack_banded(oracle_mod, n):
    a, b, c, d = workloads.random_system(n, 99, "herm")
    ab = np.zeros((3, n), np.complex128)
    ab[0, 1:] = c[:-1]
    ab[1, :] = a
    ab[2, :-1] = b[1:]
    ref = scipy.linalg.solve_banded((1, 1), ab, d)  # LAPACK zgbsv
    x = oracle_mod.thomas(a, b, c, d)
    assert rel(x, ref) <= 1e-13


def test_thomas_single_row(oracle_mod):
    a = np.array([2 - 1j])
    d = np.array([3 + 4j])
    np.testing.assert_allclose(oracle_mod.thomas(a, a * 0, a * 0, d), d / a, rtol=0, atol=1e-16)


def test_thomas_reports_zero_pivot(oracle_mod):
    a = np.array([0j, 1, 1])
    b = np.zeros(3, complex)
    c = np.zeros(3, complex)
    with pytest.raises(oracle_mod.OracleBreakdown):
        oracle_mod.thomas(a, b, c, np.ones(3, complex))


def test_thomas_batched_equals_single(oracle_mod):
    offs = np.array([0, 5, 6, 40, 41, 100])
    a, b, c, d = workloads.random_system(100, 5, "dd")
    x = oracle_mod.thomas_batched(offs, a, b, c, d, nthreads=4)
    for s in range(5):
        o0, o1 = offs[s], offs[s + 1]
        ref = np.linalg.solve(dense(a[o0:o1], b[o0:o1], c[o0:o1]), d[o0:o1])
        assert rel(x[o0:o1], ref) <= 1e-13


# --------------------------------------------------------------- CN assembly (O1, O2)
def hamiltonian_dense(V, dx):
    """H = -1/2 d^2/dx^2 + V with the 3-point stencil and Dirichlet walls, built as a dense
    matrix from the second-difference operator (independent of the oracle's formulas)."""
    n = V.shape[0]
    D2 = (np.diag(np.full(n - 1, 1.0), -1) - 2 * np.eye(n) + np.diag(np.full(n - 1, 1.0), 1))
    return -0.5 * D2 / dx**2 + np.diag(V)


@pytest.mark.parametrize("with_field", [False, True])
def test_cn_coeffs_and_rhs_match_dense_hamiltonian(oracle_mod, with_field):
    n, dx, dt = 12, 0.3, 0.05
    inp = workloads.random_cn(n, 21, dx, dt)
    xg = workloads.grid_1d(n, dx) if with_field else None
    E = 0.37 if with_field else 0.0
    Veff = inp["V"] + (xg * E if with_field else 0.0)
    H = hamiltonian_dense(Veff, dx)
    A = np.eye(n) + 0.5j * dt * H
    B = np.eye(n) - 0.5j * dt * H
    a, b, c = oracle_mod.cn_coeffs(inp["V"], dx, dt, xg, E)
    np.testing.assert_allclose(dense(a, b, c), A, rtol=0, atol=1e-14)
    assert b[0] == 0 and c[-1] == 0
    d = oracle_mod.cn_rhs(inp["psi"], inp["V"], dx, dt, xg, E)
    np.testing.assert_allclose(d, B @ inp["psi"], rtol=0, atol=1e-13)
    step = oracle_mod.cn_step(inp["psi"], inp["V"], dx, dt, xg, E)
    assert rel(step, np.linalg.solve(A, B @ inp["psi"])) <= 1e-13


# -------------------------------------------------------- CN closed form and invariants
@pytest.mark.parametrize("V0", [0.0, -0.7])
def test_cn_phase_on_sine_modes(oracle_mod, V0):
    """With constant V, sin(k pi j/(N+1)) is an eigenvector of the discrete H with
    eigenvalue (1 - cos(k pi/(N+1)))/dx^2 + V0; each CN step multiplies it by
    (1 - i lam tau)/(1 + i lam tau)."""
    N, dx, dt, steps = 257, 0.1, 0.02, 40
    j = np.arange(1, N + 1)
    tau = dt / 2
    ks = [1, 2, 7, 100, 256]
    coef = np.array([1.0, 0.5 - 0.25j, 0.3j, 0.2, -0.1])
    psi0 = sum(ck * np.sin(k * np.pi * j / (N + 1)) for k, ck in zip(ks, coef))
    out = oracle_mod.cn_propagate(psi0, np.full(N, V0), dx, dt, steps)
    ref = np.zeros(N, np.complex128)
    for k, ck in zip(ks, coef):
        lam = (1 - np.cos(k * np.pi / (N + 1))) / dx**2 + V0
        ph = (1 - 1j * lam * tau) / (1 + 1j * lam * tau)
        ref += ck * ph**steps * np.sin(k * np.pi * j / (N + 1))
    assert rel(out, ref) <= 1e-12


def test_cn_norm_conservation(oracle_mod):
    w = workloads.plain_1d(n=2048)
    out = oracle_mod.cn_propagate(w["psi0"], w["V"], w["dx"], w["dt"], 50)
    n0 = np.sum(np.abs(w["psi0"]) ** 2) * w["dx"]
    n1 = np.sum(np.abs(out) ** 2) * w["dx"]
    assert abs(n1 - n0) <= 1e-12


def test_cn_time_reversal(oracle_mod):
    inp = workloads.random_cn(500, 4)
    fwd = oracle_mod.cn_step(inp["psi"], inp["V"], inp["dx"], inp["dt"])
    back = oracle_mod.cn_step(fwd, inp["V"], inp["dx"], -inp["dt"])
    assert rel(back, inp["psi"]) <= 1e-13


def test_cn_conjugation_symmetry(oracle_mod):
    inp = workloads.random_cn(300, 6)
    lhs = np.conj(oracle_mod.cn_step(np.conj(inp["psi"]), inp["V"], inp["dx"], inp["dt"]))
    rhs = oracle_mod.cn_step(inp["psi"], inp["V"], inp["dx"], -inp["dt"])
    assert rel(lhs, rhs) <= 1e-13


def test_cn_second_order_in_dt(oracle_mod):
    """Global error of CN against the exact exponential is O(dt^2) (Sec. 2)."""
    n, dx, T = 64, 0.2, 0.4
    inp = workloads.random_cn(n, 8, dx)
    H = hamiltonian_dense(inp["V"], dx)
    w, U = np.linalg.eigh(H)
    exact = U @ (np.exp(-1j * w * T) * (U.conj().T @ inp["psi"]))
    errs = []
    for steps in (40, 80):
        out = oracle_mod.cn_propagate(inp["psi"], inp["V"], dx, T / steps, steps)
        errs.append(np.linalg.norm(out - exact))
    assert 3.6 <= errs[0] / errs[1] <= 4.4


def test_cn_step_batched_equals_single(oracle_mod):
    g = np.random.default_rng(3)
    lengths = np.array([3, 300, 1, 77])
    offs = np.concatenate([[0], np.cumsum(lengths)])
    V = g.uniform(-2, 0, offs[-1])
    psi = g.standard_normal(offs[-1]) + 1j * g.standard_normal(offs[-1])
    dxs = np.array([0.05, 0.1, 0.2, 0.15])
    out = oracle_mod.cn_step_batched(offs, psi, V, dxs, 0.02, nthreads=3)
    for s in range(4):
        o0, o1 = offs[s], offs[s + 1]
        ref = oracle_mod.cn_step(psi[o0:o1], V[o0:o1], dxs[s], 0.02)
        np.testing.assert_array_equal(out[o0:o1], ref)


# ------------------------------------------------------------------ ADI splitting (O5)
def test_adi_matches_kronecker_product(oracle_mod):
    """Lie split: rows (x) with V/2, then columns (y) with V/2, on a 6 x 5 grid, against
    dense operators built from the dense Hamiltonians."""
    nx, ny, dx, dy, dt = 6, 5, 0.3, 0.25, 0.04
    g = np.random.default_rng(11)
    V = g.uniform(-1, 0, (ny, nx))
    psi = g.standard_normal((ny, nx)) + 1j * g.standard_normal((ny, nx))
    out = oracle_mod.adi_step(psi, V, dx, dy, dt)
    ref = psi.copy()
    for y in range(ny):
        H = hamiltonian_dense(V[y] / 2, dx)
        ref[y] = np.linalg.solve(np.eye(nx) + 0.5j * dt * H, (np.eye(nx) - 0.5j * dt * H) @ ref[y])
    for x in range(nx):
        H = hamiltonian_dense(V[:, x] / 2, dy)
        ref[:, x] = np.linalg.solve(np.eye(ny) + 0.5j * dt * H,
                                    (np.eye(ny) - 0.5j * dt * H) @ ref[:, x])
    assert rel(out, ref) <= 1e-13


def test_adi_separable_phase(oracle_mod):
    """V = 0: sin modes in x and y pick up the product of the two 1D CN phases."""
    nx, ny, dx, dy, dt = 33, 17, 0.1, 0.2, 0.01
    kx, ky = 3, 5
    jx = np.arange(1, nx + 1)
    jy = np.arange(1, ny + 1)
    mode = np.outer(np.sin(ky * np.pi * jy / (ny + 1)), np.sin(kx * np.pi * jx / (nx + 1)))
    out = oracle_mod.adi_step(mode.astype(complex), np.zeros((ny, nx)), dx, dy, dt)
    tau = dt / 2
    lx = (1 - np.cos(kx * np.pi / (nx + 1))) / dx**2
    ly = (1 - np.cos(ky * np.pi / (ny + 1))) / dy**2
    ph = (1 - 1j * lx * tau) / (1 + 1j * lx * tau) * (1 - 1j * ly * tau) / (1 + 1j * ly * tau)
    assert rel(out, ph * mode) <= 1e-13


# ----------------------------------------------------------------------- adjoint (O6)
def test_adjoint_dot_product_identity(oracle_mod):
    a, b, c, d = workloads.random_system(50, 12, "dd")
    g = np.random.default_rng(1)
    G = g.standard_normal(50) + 1j * g.standard_normal(50)
    x = oracle_mod.thomas(a, b, c, d)
    lam, _, _, _ = oracle_mod.thomas_adjoint(a, b, c, x, G)
    # <lambda, d> = <G, T^{-1} d>
    assert abs(np.vdot(lam, d) - np.vdot(G, x)) <= 1e-12 * abs(np.vdot(G, x))


def test_adjoint_matches_torch_autograd(oracle_mod):
    torch = pytest.importorskip("torch")
    n = 24
    a, b, c, d = workloads.random_system(n, 13, "herm")
    ta = torch.tensor(a, requires_grad=True)
    tb = torch.tensor(b, requires_grad=True)
    tc = torch.tensor(c, requires_grad=True)
    td = torch.tensor(d, requires_grad=True)
    T = torch.diag(ta) + torch.diag(tb[1:], -1) + torch.diag(tc[:-1], 1)
    x = torch.linalg.solve(T, td)
    w = torch.tensor(np.random.default_rng(2).standard_normal(n) + 0j)
    loss = (torch.abs(x) ** 2 * w.real).sum() + (x.real * 0.3).sum()
    loss.backward()
    G = (2 * x * w.real + 0.3).detach().numpy()  # d loss/dRe x + i d loss/dIm x
    lam, ga, gb, gc = oracle_mod.thomas_adjoint(a, b, c, x.detach().numpy(), G)
    assert rel(lam, td.grad.numpy()) <= 1e-12
    assert rel(ga, ta.grad.numpy()) <= 1e-12
    assert rel(gb[1:], tb.grad.numpy()[1:]) <= 1e-12
    assert rel(gc[:-1], tc.grad.numpy()[:-1]) <= 1e-12


def _propagate_torch(torch, psi0, V, dx, dt, steps, xg, E):
    n = psi0.shape[0]
    D2 = (torch.diag(torch.ones(n - 1, dtype=torch.float64), -1) - 2 * torch.eye(n, dtype=torch.float64)
          + torch.diag(torch.ones(n - 1, dtype=torch.float64), 1))
    psi = psi0
    for k in range(steps):
        H = (-0.5 * D2 / dx**2 + torch.diag(V + xg * E[k])).to(torch.complex128)
        A = torch.eye(n, dtype=torch.complex128) + 0.5j * dt * H
        B = torch.eye(n, dtype=torch.complex128) - 0.5j * dt * H
        psi = torch.linalg.solve(A, B @ psi)
    return psi


def test_propagate_grad_matches_dense_autograd(oracle_mod):
    torch = pytest.importorskip("torch")
    n, dx, dt, steps = 32, 0.4, 0.05, 12
    g = np.random.default_rng(5)
    x = workloads.grid_1d(n, dx)
    V = workloads.softcore(x)
    E = g.normal(0, 0.05, steps)
    psi0 = workloads.gaussian(x, 0.0, 2.0, 1.0, dx)
    phi = workloads.gaussian(x, 1.0, 1.5, 0.8, dx)
    tV = torch.tensor(V, requires_grad=True)
    tE = torch.tensor(E, requires_grad=True)
    tpsi = torch.tensor(psi0, requires_grad=True)
    out = _propagate_torch(torch, tpsi, tV, dx, dt, steps, torch.tensor(x), tE)
    ov = (torch.conj(torch.tensor(phi)) * out).sum() * dx
    loss = torch.abs(ov) ** 2
    loss.backward()
    psiT = oracle_mod.cn_propagate(psi0, V, dx, dt, steps, x, E)
    ovn = np.sum(np.conj(phi) * psiT) * dx
    G_T = 2 * ovn * phi * dx  # d|<phi|psi>|^2 / dRe psi + i d/dIm psi
    gpsi0, dV, dE = oracle_mod.cn_propagate_grad(psi0, V, dx, dt, steps, G_T, x, E)
    assert rel(dV, tV.grad.numpy()) <= 1e-10
    assert rel(dE, tE.grad.numpy()) <= 1e-10
    assert rel(gpsi0, tpsi.grad.numpy()) <= 1e-10


def test_propagate_grad_matches_finite_differences(oracle_mod):
    n, dx, dt, steps = 40, 0.3, 0.04, 10
    g = np.random.default_rng(9)
    x = workloads.grid_1d(n, dx)
    V = workloads.softcore(x)
    E = g.normal(0, 0.05, steps)
    psi0 = workloads.gaussian(x, 0.0, 2.0, 1.0, dx)
    phi = workloads.gaussian(x, 1.0, 1.5, 0.8, dx)

    def loss(Vv, Ev):
        p = oracle_mod.cn_propagate(psi0, Vv, dx, dt, steps, x, Ev)
        return abs(np.sum(np.conj(phi) * p) * dx) ** 2

    psiT = oracle_mod.cn_propagate(psi0, V, dx, dt, steps, x, E)
    G_T = 2 * (np.sum(np.conj(phi) * psiT) * dx) * phi * dx
    _, dV, dE = oracle_mod.cn_propagate_grad(psi0, V, dx, dt, steps, G_T, x, E)
    h = 1e-5
    for j in (3, 17, 20, 33):
        Vp, Vm = V.copy(), V.copy()
        Vp[j] += h
        Vm[j] -= h
        fd = (loss(Vp, E) - loss(Vm, E)) / (2 * h)
        assert abs(fd - dV[j]) <= 1e-7 * max(abs(fd), 1e-3)
    for k in (0, 4, 9):
        Ep, Em = E.copy(), E.copy()
        Ep[k] += h
        Em[k] -= h
        fd = (loss(V, Ep) - loss(V, Em)) / (2 * h)
        assert abs(fd - dE[k]) <= 1e-7 * max(abs(fd), 1e-3)


# ------------------------------------------- absorbing (non-Hermitian) potential V - iW
def test_absorbing_coeffs_and_rhs_match_dense_hamiltonian(oracle_mod):
    """With H = -1/2 D2 + diag(V - iW), the step is (1 + i tau H)^{-1} (1 - i tau H) psi; the
    right side is 1 - i tau H, which differs from T^dagger once W is nonzero."""
    n, dx, dt = 12, 0.3, 0.05
    inp = workloads.random_cn(n, 23, dx, dt)
    W = np.random.default_rng(5).uniform(0.0, 3.0, n)
    H = hamiltonian_dense(inp["V"], dx) - 1j * np.diag(W)
    A = np.eye(n) + 0.5j * dt * H
    B = np.eye(n) - 0.5j * dt * H
    a, b, c = oracle_mod.cn_coeffs(inp["V"], dx, dt, W=W)
    np.testing.assert_allclose(dense(a, b, c), A, rtol=0, atol=1e-14)
    d = oracle_mod.cn_rhs(inp["psi"], inp["V"], dx, dt, W=W)
    np.testing.assert_allclose(d, B @ inp["psi"], rtol=0, atol=1e-13)
    assert np.max(np.abs(B - A.conj().T)) > 0.01  # T^dagger would be a different operator
    step = oracle_mod.cn_step(inp["psi"], inp["V"], dx, dt, W=W)
    assert rel(step, np.linalg.solve(A, B @ inp["psi"])) <= 1e-13


@pytest.mark.parametrize("W0", [0.05, 1.5])
def test_absorbing_amplification_on_sine_modes(oracle_mod, W0):
    """With constant V0 and W0 the sine modes stay eigenvectors of H, with eigenvalue
    lam - i W0; one step multiplies each by (1 - tau W0 - i tau lam)/(1 + tau W0 + i tau lam),
    whose modulus is below one."""
    N, dx, dt, steps, V0 = 257, 0.1, 0.02, 40, -0.4
    j = np.arange(1, N + 1)
    tau = dt / 2
    ks = [1, 3, 50, 256]
    coef = np.array([1.0, 0.4j, -0.3 + 0.2j, 0.1])
    psi0 = sum(ck * np.sin(k * np.pi * j / (N + 1)) for k, ck in zip(ks, coef))
    out = oracle_mod.cn_propagate(psi0, np.full(N, V0), dx, dt, steps, W=np.full(N, W0))
    ref = np.zeros(N, np.complex128)
    for k, ck in zip(ks, coef):
        lam = (1 - np.cos(k * np.pi / (N + 1))) / dx**2 + V0
        g = (1 - tau * W0 - 1j * tau * lam) / (1 + tau * W0 + 1j * tau * lam)
        assert abs(g) < 1
        ref += ck * g**steps * np.sin(k * np.pi * j / (N + 1))
    assert rel(out, ref) <= 1e-12


def test_absorbing_norm_decays_and_zero_W_is_hermitian_step(oracle_mod):
    """W >= 0 makes every step contract the norm; W = 0 gives the Hermitian step exactly."""
    w = workloads.absorbing_1d(n=2048)
    psi = workloads.gaussian(w["x"], w["x"][1880], 5.0, 2.0, w["dx"])  # on the ramp
    norms = [np.sum(np.abs(psi) ** 2)]
    for _ in range(30):
        psi = oracle_mod.cn_step(psi, w["V"], w["dx"], w["dt"], W=w["W"])
        norms.append(np.sum(np.abs(psi) ** 2))
    assert all(b < a for a, b in zip(norms, norms[1:]))
    z = oracle_mod.cn_step(psi, w["V"], w["dx"], w["dt"], W=np.zeros(2048))
    h = oracle_mod.cn_step(psi, w["V"], w["dx"], w["dt"])
    assert np.array_equal(z, h)


def test_absorbing_loss_rate(oracle_mod):
    """For small dt the norm falls at the rate d|psi|^2/dt = -2 sum W |psi|^2."""
    w = workloads.absorbing_1d(n=2048)
    psi0 = w["psi0"]
    W = np.full(2048, 0.3)
    for dt in (1e-3, 5e-4):
        p1 = oracle_mod.cn_step(psi0, w["V"], w["dx"], dt, W=W)
        rate = (np.sum(np.abs(p1) ** 2) - np.sum(np.abs(psi0) ** 2)) / dt
        expect = -2 * np.sum(W * np.abs(psi0) ** 2)
        assert abs(rate - expect) <= 2 * dt * abs(expect)


def test_absorbing_pin_rejects_t_dagger_right_side(oracle_mod):
    """The plausible mistake of keeping T^dagger as the right side (1 + tau W - i tau H0) gives
    a norm-preserving step; the amplification pin above tells it apart by far."""
    N, dx, dt, V0, W0 = 257, 0.1, 0.02, -0.4, 1.5
    j = np.arange(1, N + 1)
    tau = dt / 2
    k = 3
    mode = np.sin(k * np.pi * j / (N + 1)).astype(np.complex128)
    V, W = np.full(N, V0), np.full(N, W0)
    a, b, c = oracle_mod.cn_coeffs(V, dx, dt, W=W)
    wrong = oracle_mod.thomas(a, b, c, oracle_mod.cn_rhs(mode, V, dx, dt, W=-W))
    right = oracle_mod.cn_step(mode, V, dx, dt, W=W)
    lam = (1 - np.cos(k * np.pi / (N + 1))) / dx**2 + V0
    g = (1 - tau * W0 - 1j * tau * lam) / (1 + tau * W0 + 1j * tau * lam)
    assert rel(right, g * mode) <= 1e-13
    assert rel(wrong, g * mode) > 1e-3
    assert abs(np.linalg.norm(wrong) - np.linalg.norm(mode)) <= 1e-12 * np.linalg.norm(mode)


def _propagate_torch_w(torch, psi0, V, W, dx, dt, steps, xg, E):
    """Dense restatement of the absorbing step: H = -1/2 D2 + diag(V + x E_k - i W)."""
    n = psi0.shape[0]
    D2 = (torch.diag(torch.ones(n - 1, dtype=torch.float64), -1) - 2 * torch.eye(n, dtype=torch.float64)
          + torch.diag(torch.ones(n - 1, dtype=torch.float64), 1))
    psi = psi0
    for k in range(steps):
        H = (-0.5 * D2 / dx**2 + torch.diag(V + xg * E[k])).to(torch.complex128) \
            - 1j * torch.diag(W).to(torch.complex128)
        A = torch.eye(n, dtype=torch.complex128) + 0.5j * dt * H
        B = torch.eye(n, dtype=torch.complex128) - 0.5j * dt * H
        psi = torch.linalg.solve(A, B @ psi)
    return psi


def test_absorbing_propagate_grad_matches_dense_autograd(oracle_mod):
    """Reverse mode with an absorbing potential: lambda = T^{-H} G and G_k = B^H lambda with
    B = 1 - i tau H != T^H; pinned to torch autograd through dense non-Hermitian steps."""
    torch = pytest.importorskip("torch")
    n, dx, dt, steps = 32, 0.4, 0.05, 12
    g = np.random.default_rng(15)
    x = workloads.grid_1d(n, dx)
    V = workloads.softcore(x)
    W = workloads.absorber(n, frac=0.25, strength=3.0)
    E = g.normal(0, 0.05, steps)
    psi0 = workloads.gaussian(x, 2.0, 2.0, 1.5, dx)
    phi = workloads.gaussian(x, 3.0, 1.5, 0.8, dx)
    tV = torch.tensor(V, requires_grad=True)
    tE = torch.tensor(E, requires_grad=True)
    tpsi = torch.tensor(psi0, requires_grad=True)
    out = _propagate_torch_w(torch, tpsi, tV, torch.tensor(W), dx, dt, steps, torch.tensor(x), tE)
    loss = torch.abs((torch.conj(torch.tensor(phi)) * out).sum() * dx) ** 2
    loss.backward()
    psiT = oracle_mod.cn_propagate(psi0, V, dx, dt, steps, x, E, W=W)
    assert rel(psiT, out.detach().numpy()) <= 1e-12
    G_T = 2 * (np.sum(np.conj(phi) * psiT) * dx) * phi * dx
    gpsi0, dV, dE = oracle_mod.cn_propagate_grad(psi0, V, dx, dt, steps, G_T, x, E, W=W)
    assert rel(dV, tV.grad.numpy()) <= 1e-10
    assert rel(dE, tE.grad.numpy()) <= 1e-10
    assert rel(gpsi0, tpsi.grad.numpy()) <= 1e-10
    # the Hermitian recursion G_k = T_k lambda_k is wrong here: it must miss the pin
    g_herm, _, _ = oracle_mod.cn_propagate_grad(psi0, V, dx, dt, steps, G_T, x, E, W=None)
    assert rel(g_herm, tpsi.grad.numpy()) > 1e-3


def test_absorbing_propagate_grad_matches_finite_differences(oracle_mod):
    n, dx, dt, steps = 40, 0.3, 0.04, 10
    g = np.random.default_rng(19)
    x = workloads.grid_1d(n, dx)
    V = workloads.softcore(x)
    W = workloads.absorber(n, frac=0.3, strength=2.0)
    E = g.normal(0, 0.05, steps)
    psi0 = workloads.gaussian(x, 2.0, 2.0, 1.0, dx)
    phi = workloads.gaussian(x, 1.0, 1.5, 0.8, dx)

    def loss(Vv, Ev):
        p = oracle_mod.cn_propagate(psi0, Vv, dx, dt, steps, x, Ev, W=W)
        return abs(np.sum(np.conj(phi) * p) * dx) ** 2

    psiT = oracle_mod.cn_propagate(psi0, V, dx, dt, steps, x, E, W=W)
    G_T = 2 * (np.sum(np.conj(phi) * psiT) * dx) * phi * dx
    _, dV, dE = oracle_mod.cn_propagate_grad(psi0, V, dx, dt, steps, G_T, x, E, W=W)
    h = 1e-5
    for j in (3, 17, 20, 33, 38):
        Vp, Vm = V.copy(), V.copy()
        Vp[j] += h
        Vm[j] -= h
        fd = (loss(Vp, E) - loss(Vm, E)) / (2 * h)
        assert abs(fd - dV[j]) <= 1e-7 * max(abs(fd), 1e-3)
    for k in (0, 4, 9):
        Ep, Em = E.copy(), E.copy()
        Ep[k] += h
        Em[k] -= h
        fd = (loss(V, Ep) - loss(V, Em)) / (2 * h)
        assert abs(fd - dE[k]) <= 1e-7 * max(abs(fd), 1e-3)


def test_absorbing_propagate_grad_without_w_is_the_hermitian_recursion(oracle_mod):
    """W = 0 gives the real-potential recursion G_k = T_k lambda_k, pinned above."""
    n, dx, dt, steps = 30, 0.3, 0.04, 6
    x = workloads.grid_1d(n, dx)
    V = workloads.softcore(x)
    psi0 = workloads.gaussian(x, 0.0, 2.0, 1.0, dx)
    G_T = workloads.complex_normal(np.random.default_rng(3), n)
    a = oracle_mod.cn_propagate_grad(psi0, V, dx, dt, steps, G_T, x, np.zeros(steps))
    b = oracle_mod.cn_propagate_grad(psi0, V, dx, dt, steps, G_T, x, np.zeros(steps),
                                     W=np.zeros(n))
    for u, v in zip(a, b):
        assert rel(u, v) <= 1e-15


# --------------------------------------------------- partial-wave (radial) step, Sec. 3
def _legendre_cos_matrix(l0, nl):
    """<Y_l0|cos(theta)|Y_l'0> for l, l' = l0 .. l0+nl-1 by Gauss-Legendre quadrature of the
    normalised Legendre polynomials (independent of any closed form)."""
    from numpy.polynomial import legendre

    xq, wq = legendre.leggauss(2 * (l0 + nl) + 4)
    P = np.array([legendre.legval(xq, np.eye(l0 + nl)[l]) * np.sqrt((2 * l + 1) / 2.0)
                  for l in range(l0, l0 + nl)])
    return (P * wq * xq) @ P.T


def _dense_cn(H, dt, psi):
    n = H.shape[0]
    return np.linalg.solve(np.eye(n) + 0.5j * dt * H, (np.eye(n) - 0.5j * dt * H) @ psi)


@pytest.mark.parametrize("l0,nl", [(0, 1), (0, 5), (3, 4)])
def test_radial_step_matches_dense_split(oracle_mod, l0, nl):
    """The partial-wave step against a dense restatement: H_l = -1/2 D2 + V + l(l+1)/(2 r^2)
    per wave (D2 the second-difference matrix), then H_E = E r C across waves with C from
    quadrature, each applied as a dense CN step."""
    nr, dr, dt, E = 24, 0.25, 0.05, 0.7
    g = np.random.default_rng(l0 + 10 * nl)
    r = dr * np.arange(1, nr + 1)
    V = -1.0 / np.sqrt(r * r + 1.0)
    psi = workloads.complex_normal(g, nl * nr)
    got = oracle_mod.radial_step(psi, V, dr, dt, E, l0, nl)
    ref = psi.reshape(nl, nr).copy()
    for k in range(nl):
        l = l0 + k
        H = hamiltonian_dense(V + l * (l + 1) / (2 * r * r), dr)
        ref[k] = _dense_cn(H, dt, ref[k])
    C = _legendre_cos_matrix(l0, nl)
    for j in range(nr):
        ref[:, j] = _dense_cn(E * r[j] * C, dt, ref[:, j])
    assert rel(got, ref.ravel()) <= 1e-13
    # both halves are unitary: the norm is kept
    assert abs(np.linalg.norm(got) / np.linalg.norm(psi) - 1) <= 1e-13


def test_radial_single_wave_without_field_is_the_1d_step(oracle_mod):
    nr, dr, dt = 500, 0.1, 0.02
    g = np.random.default_rng(2)
    V = g.uniform(-1, 0, nr)
    psi = workloads.complex_normal(g, nr)
    got = oracle_mod.radial_step(psi, V, dr, dt, 0.3, 0, 1)
    np.testing.assert_array_equal(got, oracle_mod.cn_step(psi, V, dr, dt))


def test_legendre_quadrature_pin_is_tridiagonal(oracle_mod):
    """The quadrature matrix is the tridiagonal coupling the radial step uses: zero off the
    first off-diagonals, symmetric, and the known closed form there."""
    C = _legendre_cos_matrix(0, 8)
    off = np.array([(l + 1) / np.sqrt((2 * l + 1) * (2 * l + 3)) for l in range(7)])
    assert np.allclose(np.diag(C, 1), off, atol=1e-14)
    assert np.allclose(C - np.diag(np.diag(C, 1), 1) - np.diag(np.diag(C, 1), -1), 0, atol=1e-14)
