"""GPU parity at the benchmark's full sizes, in the launch configurations bench.py times:

* one Lie-split ADI step of the 4096 x 4096 grid (x-sweep over 4096 contiguous lines, y-sweep
  over 4096 interleaved lines, V/2 each), against the oracle's ADI step of the whole grid;
* the 2^28-unknown explicit solve with the automatic plan, checked by a property that holds at
  any size (the relative residual of T x = d, computed on the device with plain tensor ops),
  since the oracle's serial solve of 2^28 rows is out of reach of a test;
* one CN step of the whole uneven batch (10^4 systems), system by system against the oracle;
* one 2^22-row matrix with 16 right-hand sides, each against the oracle.

Tolerances: relative L2 <= 1e-11 for the ADI state (FP64 on both sides; rounding only); relative
residual <= 1e-13 for the solve (backward-stable elimination of a diagonally dominant system).
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


def test_large_system_2e28_residual(gpu):
    torch, cn = gpu
    log("2^28 solve")
    N = 1 << 28
    g = torch.Generator(device="cuda")
    g.manual_seed(1002)
    V = torch.rand(N, dtype=torch.float64, device="cuda", generator=g) - 1.0
    a, b, c = cn.assemble(V, 0.01, 0.02)
    del V
    d = torch.empty(N, dtype=torch.complex128, device="cuda")
    d.real.normal_(generator=g)
    d.imag.normal_(generator=g)
    x = cn.solve(a, b, c, d, layout=cn.Layout.contiguous(N, 1))
    r = a * x
    r[1:] += b[1:] * x[:-1]
    r[:-1] += c[:-1] * x[1:]
    r -= d
    resid = float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(d))
    del r, a, b, c, d
    finite = bool(torch.isfinite(x).all())
    del x
    torch.cuda.empty_cache()
    assert finite
    assert resid <= 1e-13
    assert cn.get_status() == 0


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
