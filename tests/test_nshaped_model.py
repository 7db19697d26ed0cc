"""The reading of Table 1 / Appendix I (CPU model) against the oracle, no GPU.

Pins the readings of the printed stages: r_i in RD, joint-line neighbours in RS, the
(RD+JD)+(RU+JU) order, blocks without interior rows, two-slot joins and nesting (Eq. (6)).
"""
import itertools

import numpy as np
import pytest

import workloads
from oracle import nshaped_model as nm


def rel(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 7, 10])
def test_every_joint_line_subset(oracle_mod, n):
    a, b, c, d = workloads.random_system(n, 100 + n, "dd")
    ref = oracle_mod.thomas(a, b, c, d)
    inner = list(range(1, n - 1))
    for k in range(len(inner) + 1):
        for sub in itertools.combinations(inner, k):
            J = [0, *sub, n - 1]
            assert rel(nm.solve(a, b, c, d, J), ref) <= 1e-13, J


def test_stage_orders_agree_bitwise():
    a, b, c, d = workloads.random_system(200, 3, "herm")
    J = nm.uniform_joints(200, 13)
    x1 = nm.solve(a, b, c, d, J, order="RD+JD,RU+JU")
    x2 = nm.solve(a, b, c, d, J, order="RD+RU,JU+JD")
    np.testing.assert_array_equal(x1, x2)


@pytest.mark.parametrize("p", [1, 2, 3, 8, 64, 5000])
def test_uniform_partitions(oracle_mod, p):
    a, b, c, d = workloads.random_system(4097, 7, "herm")
    x = nm.solve(a, b, c, d, nm.uniform_joints(4097, p))
    assert rel(x, oracle_mod.thomas(a, b, c, d)) <= 1e-13


def test_random_uneven_joints(oracle_mod):
    g = np.random.default_rng(4)
    n = 20000
    a, b, c, d = workloads.random_system(n, 8, "dd")
    inner = np.sort(g.choice(np.arange(1, n - 1), 700, replace=False))
    J = [0, *inner.tolist(), n - 1]
    assert rel(nm.solve(a, b, c, d, J), oracle_mod.thomas(a, b, c, d)) <= 1e-13


@pytest.mark.parametrize("depth", [1, 2, 3, 4])
def test_nested_levels(oracle_mod, depth):
    n = 6000
    a, b, c, d = workloads.random_system(n, 9, "herm")
    J = nm.uniform_joints(n, 7)
    nested = []
    m = len(J)
    for _ in range(depth - 1):
        Jn = nm.uniform_joints(m, 5)
        nested.append(Jn)
        m = len(Jn)
    x = nm.solve(a, b, c, d, J, nested)
    assert rel(x, oracle_mod.thomas(a, b, c, d)) <= 1e-13


def test_cn_pivots_have_real_part_at_least_one(oracle_mod):
    """T = I + iK with K real symmetric: every Schur-complement pivot has Re >= 1."""
    w = workloads.plain_1d(n=3000)
    a, b, c = oracle_mod.cn_coeffs(w["V"], w["dx"], w["dt"])
    d = oracle_mod.cn_rhs(w["psi0"], w["V"], w["dx"], w["dt"])
    J = nm.uniform_joints(3000, 37)
    x, piv = nm.solve(a, b, c, d, J, [nm.uniform_joints(len(J), 4)], return_pivots=True)
    assert min(np.real(piv)) >= 1.0 - 1e-12
    assert rel(x, oracle_mod.thomas(a, b, c, d)) <= 1e-13


@pytest.mark.parametrize("m", [1, 2, 3, 4, 8, 17])
@pytest.mark.parametrize("kind", ["dd", "herm", "cn"])
def test_rd_form_slots_equal_table1_stages(oracle_mod, m, kind):
    """The RD form of one block (RD, JD, the forward sum standing for RU, JU) produces the same
    two joint rows as Table 1's four stages on that block, and its substitution along the RD
    rows gives the interior solution."""
    n = m + 1
    if kind == "cn":
        w = workloads.plain_1d(n=n)
        a, b, c = oracle_mod.cn_coeffs(w["V"], w["dx"], w["dt"])
        d = oracle_mod.cn_rhs(w["psi0"], w["V"], w["dx"], w["dt"])
    else:
        a, b, c, d = workloads.random_system(n, 500 + m, kind)
    b = np.array(b, np.complex128)
    c = np.array(c, np.complex128)
    b[0] = 0.0
    c[-1] = 0.0
    ra, rb, rc, rd_, _ = nm._stages_one_level(np.array(a, np.complex128), b.copy(), c.copy(),
                                              np.array(d, np.complex128), [0, m])
    UA, UC, UD, DB, DA, DD, delta = nm.rd_form_block(a, b, c, d)
    scale = np.max(np.abs([ra[0], rc[0], rd_[0], rb[1], ra[1], rd_[1]]))
    got = np.array([UA, UC, UD, DB, a[m] + DA, d[m] + DD])
    want = np.array([ra[0], rc[0], rd_[0], rb[1], ra[1], rd_[1]])
    assert np.max(np.abs(got - want)) <= 1e-13 * scale
    # the 2x2 joint system, then the interior rows by substitution along the RD rows
    M2 = np.array([[UA, UC], [DB, a[m] + DA]])
    psiJK = np.linalg.solve(M2, np.array([UD, d[m] + DD]))
    psi = nm.rd_form_substitute(a, b, c, delta, psiJK[0], psiJK[1])
    ref = oracle_mod.thomas(a, b, c, d)
    assert rel(psi, ref) <= 1e-13


@pytest.mark.parametrize("n,p", [(37, 8), (200, 13), (1000, 64)])
def test_deferred_joint_row_term(oracle_mod, n, p):
    """Cross-step fusion defers, in every tile's joint row J, the explicit half-step's term
    i kap psi_{J-1} (the left neighbour lies in another tile) to the reduced system.  Pins that
    deferral: RD, RU, JD and JU never touch d at a joint row, so the reduced matrix is unchanged
    and the reduced right-hand side differs by exactly i kap psi_{J-1} at every joint line
    w >= 1; adding it back there and substituting gives the oracle's CN step."""
    dx, dt = 0.1, 0.02
    inp = workloads.random_cn(n, 300 + n, dx, dt)
    psi, V = inp["psi"], inp["V"]
    a, b, c = oracle_mod.cn_coeffs(V, dx, dt)
    d = oracle_mod.cn_rhs(psi, V, dx, dt)
    kap = dt / (4.0 * dx * dx)  # the off-diagonal magnitude, |b| = |c| = kap
    assert np.allclose(np.abs(b[1:]), kap, rtol=1e-14, atol=0)
    J = nm.uniform_joints(n, p)
    deferred = np.zeros(len(J), np.complex128)
    dp = d.copy()
    for w in range(1, len(J)):
        deferred[w] = 1j * kap * psi[J[w] - 1]
        dp[J[w]] -= deferred[w]

    def stages(dd):
        aa, bb, cc = np.array(a), np.array(b), np.array(c)
        bb[0] = 0.0
        cc[-1] = 0.0
        ddd = np.array(dd)
        out = nm._stages_one_level(aa, bb, cc, ddd, J)
        return out, (aa, bb, cc, ddd)

    (ra, rb, rc, rd_full, _), _ = stages(d)
    (ra2, rb2, rc2, rd_part, _), (aa, bb, cc, ddd) = stages(dp)
    assert np.array_equal(ra, ra2) and np.array_equal(rb, rb2) and np.array_equal(rc, rc2)
    scale = np.max(np.abs(rd_full))
    assert np.max(np.abs(rd_full - (rd_part + deferred))) <= 1e-14 * scale
    # the fused reading end to end: reduced system with the deferred terms, then SS on the
    # interior rows that the partial right-hand side produced
    support = nm._rs(ra2, rb2, rc2, rd_part + deferred, [])
    x = np.empty(n, np.complex128)
    x[np.asarray(J)] = support
    nm._ss(aa, bb, cc, ddd, J, support, x)
    assert rel(x, oracle_mod.cn_step(psi, V, dx, dt)) <= 1e-12
    # a deferred term with the wrong neighbour does not pass
    wrong = deferred.copy()
    for w in range(1, len(J)):
        wrong[w] = 1j * kap * psi[J[w] - 2]
    bad = nm._rs(ra2, rb2, rc2, rd_part + wrong, [])
    assert rel(bad, support) > 1e-6


def test_absorbing_pivots_and_nested_solve(oracle_mod):
    """With an absorbing potential T = I + tau W + iK (W >= 0 diagonal, K real symmetric) the
    Hermitian part of T is at least I, and so is that of every Schur complement: every pivot of
    the partitioned elimination keeps Re >= 1 (no pivoting needed, as for the Hermitian case),
    and the nested N-shaped solve equals the oracle's Thomas solve."""
    w = workloads.absorbing_1d(n=3000)
    a, b, c = oracle_mod.cn_coeffs(w["V"], w["dx"], w["dt"], W=w["W"])
    d = oracle_mod.cn_rhs(w["psi0"], w["V"], w["dx"], w["dt"], W=w["W"])
    assert max(np.real(a)) > 1.0 + 1e-3  # the absorber really changes the diagonal
    J = nm.uniform_joints(3000, 37)
    x, piv = nm.solve(a, b, c, d, J, [nm.uniform_joints(len(J), 4)], return_pivots=True)
    assert min(np.real(piv)) >= 1.0 - 1e-12
    assert rel(x, oracle_mod.thomas(a, b, c, d)) <= 1e-13
