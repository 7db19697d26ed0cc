"""Literal CPU model of the N-shaped partition method -- TEST INFRASTRUCTURE ONLY.

The oracle proper is the plain elimination in ``cn_oracle.c``.  This module restates the
stages of Table 1 (arXiv 2205.00856, Sec. 4.1) one row operation at a time, over an arbitrary
set of joint lines and with nesting (Sec. 4.1.6, Eq. (6)), so that tests can check the reading
of the paper's stages against the oracle on tiny systems (every joint-line subset) without
involving the GPU.  It shares nothing with the HIP path.

Notation follows the paper, rows 0-based: b_i = T[i, i-1], a_i = T[i, i], c_i = T[i, i+1];
joint lines J_0 = 0 < J_1 < ... < J_nbl = n-1; block w spans J_w .. J_{w+1}.

Readings taken where the printed table is ambiguous:
  * RD writes "a_i + r c_{i-1}" with a bare r: it is r_i.
  * RS writes rows i-1 / i+1: they are the neighbouring joint lines J_{w-1} / J_{w+1}.
  * The caption says JU and RU commute; JU needs the RU-reduced row J_w+1, so it is JD and RU
    that commute.  The model runs (RD+JD)+(RU+JU) (Sec. 5.2.1) by default and can run
    (RD+RU)+(JU+JD) to show both orders give the same numbers.
  * A block without interior rows (J_{w+1} = J_w + 1) skips RD/RU/JU/JD: its joint rows are
    already coupled directly.
  * The "atomic" additions to a_{J_w}, d_{J_w} use two slots per joint line (Sec. 4.1.3,
    distributed-memory variant), summed in a fixed order: own value + JD slot + JU slot.
"""
from __future__ import annotations

import numpy as np


def _stages_one_level(a, b, c, d, J, order="RD+JD,RU+JU"):
    """Apply RD, JD, RU, JU for every block; return the reduced joint-line system and the
    per-row state needed by SS.  Arrays are modified in place (they are copies)."""
    n = a.shape[0]
    nbl = len(J) - 1
    slot_jd_a = np.zeros(nbl + 1, np.complex128)
    slot_jd_d = np.zeros(nbl + 1, np.complex128)
    slot_ju_a = np.zeros(nbl + 1, np.complex128)
    slot_ju_d = np.zeros(nbl + 1, np.complex128)
    pivots = []

    def rd(w):
        for i in range(J[w] + 2, J[w + 1]):
            pivots.append(a[i - 1])
            r = -b[i] / a[i - 1]
            b[i] = r * b[i - 1]
            a[i] = a[i] + r * c[i - 1]
            d[i] = d[i] + r * d[i - 1]

    def jd(w):
        i = J[w + 1]
        if i - J[w] < 2:
            return
        pivots.append(a[i - 1])
        r = -b[i] / a[i - 1]
        b[i] = r * b[i - 1]
        slot_jd_a[w + 1] = r * c[i - 1]
        slot_jd_d[w + 1] = r * d[i - 1]

    def ru(w):
        for i in range(J[w + 1] - 2, J[w], -1):
            pivots.append(a[i + 1])
            r = -c[i] / a[i + 1]
            b[i] = b[i] + r * b[i + 1]
            c[i] = r * c[i + 1]
            d[i] = d[i] + r * d[i + 1]

    def ju(w):
        i = J[w]
        if J[w + 1] - i < 2:
            return
        pivots.append(a[i + 1])
        r = -c[i] / a[i + 1]
        c[i] = r * c[i + 1]
        slot_ju_a[w] = r * b[i + 1]
        slot_ju_d[w] = r * d[i + 1]

    if order == "RD+JD,RU+JU":
        for w in range(nbl):
            rd(w)
            jd(w)
        for w in range(nbl):
            ru(w)
            ju(w)
    elif order == "RD+RU,JU+JD":
        for w in range(nbl):
            rd(w)
            ru(w)
        for w in range(nbl):
            ju(w)
            jd(w)
    else:
        raise ValueError(order)

    # joint-line system (Fig. 1e): row w couples J_{w-1}, J_w, J_{w+1}
    Jarr = np.asarray(J)
    ra = a[Jarr] + slot_jd_a + slot_ju_a
    rd_ = d[Jarr] + slot_jd_d + slot_ju_d
    rb = b[Jarr].copy()
    rc = c[Jarr].copy()
    rb[0] = 0.0
    rc[-1] = 0.0
    return ra, rb, rc, rd_, pivots


def _rs(a, b, c, d, pivots):
    """RS stage: serial elimination on the joint-line system (Table 1)."""
    a = a.copy()
    d = d.copy()
    m = a.shape[0]
    for i in range(1, m):
        pivots.append(a[i - 1])
        r = -b[i] / a[i - 1]
        a[i] = a[i] + r * c[i - 1]
        d[i] = d[i] + r * d[i - 1]
    psi = np.empty(m, np.complex128)
    pivots.append(a[m - 1])
    psi[m - 1] = d[m - 1] / a[m - 1]
    for i in range(m - 2, -1, -1):
        psi[i] = (d[i] - c[i] * psi[i + 1]) / a[i]
    return psi


def _ss(a, b, c, d, J, support, psi):
    """SS stage: psi_i = (d_i - b_i psi_{J_w} - c_i psi_{J_{w+1}}) / a_i for interior rows."""
    for w in range(len(J) - 1):
        for i in range(J[w] + 1, J[w + 1]):
            r = 1.0 / a[i]
            psi[i] = (d[i] - b[i] * support[w] - c[i] * support[w + 1]) * r
    return psi


def solve(a, b, c, d, J, nested=(), order="RD+JD,RU+JU", return_pivots=False):
    """Solve T x = d with the N-shaped method on joint lines J.

    ``nested`` is a sequence of joint-line sets for the reduced systems (Eq. (6)): nested[0]
    partitions the nbl+1 joint rows of this level, nested[1] those of the next, and so on.
    The innermost reduced system is solved by the serial RS stage.
    """
    a = np.array(a, np.complex128)
    b = np.array(b, np.complex128)
    c = np.array(c, np.complex128)
    d = np.array(d, np.complex128)
    n = a.shape[0]
    J = list(J)
    if J[0] != 0 or J[-1] != n - 1 or any(J[k + 1] <= J[k] for k in range(len(J) - 1)):
        raise ValueError("joint lines must start at 0, end at n-1 and increase")
    b[0] = 0.0
    c[n - 1] = 0.0
    pivots = []
    if n == 1:
        x = d / a
        return (x, [a[0]]) if return_pivots else x
    ra, rb, rc, rdd, piv = _stages_one_level(a, b, c, d, J, order)
    pivots += piv
    if nested:
        support, piv2 = solve(ra, rb, rc, rdd, nested[0], nested[1:], order, True)
        pivots += piv2
    else:
        support = _rs(ra, rb, rc, rdd, pivots)
    psi = np.empty(n, np.complex128)
    psi[np.asarray(J)] = support
    _ss(a, b, c, d, J, support, psi)
    return (psi, pivots) if return_pivots else psi


def uniform_joints(n, p):
    """J_w = w p for w < nbl and J_nbl = n-1 (blocks of p rows, the last one shorter)."""
    if n <= 1:
        return [0]
    J = list(range(0, n - 1, p))
    J.append(n - 1)
    return J


def rd_form_block(a, b, c, d):
    """One block J = 0 .. K = m of the rows (a, b, c, d), reduced the way a lane of the GPU path
    does it (the RD form):

      RD   row i = 1 .. m-1 is eliminated downwards and scaled by its pivot, giving
           psi_i + beta_i psi_J + gamma_i psi_{i+1} = delta_i   (Table 1, RD);
      JD   row K takes r = -b_K times RD row m-1 (Table 1, JD);
      RU   is needed only for JU, which uses row J+1 after RU:  psi_1 + bf psi_J + gf psi_K = df.
           Substituting the RD rows into one another gives that row as a forward sum,
           psi_1 = sum_k P_k (delta_k - beta_k psi_J) + P_m psi_K,  P_1 = 1, P_{k+1} = -gamma_k P_k,
           so bf = sum_k P_k beta_k, df = sum_k P_k delta_k, gf = -P_m;
      JU   row J takes r = -c_J times that row (Table 1, JU).

    Returns (UA, UC, UD, DB, DA, DD, delta) with
      UA psi_J + UC psi_K = UD          (row J with its own coefficients folded in),
      DB psi_J + DA psi_K = DD          (what the block adds to row K, besides row K itself),
    and the RD right-hand sides delta_1 .. delta_{m-1}."""
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    c = np.asarray(c, np.complex128)
    d = np.asarray(d, np.complex128)
    m = a.shape[0] - 1
    if m < 2:
        return a[0], c[0], d[0], b[m], 0.0, 0.0, np.zeros(0, np.complex128)
    beta = np.zeros(m, np.complex128)
    gamma = np.zeros(m, np.complex128)
    delta = np.zeros(m, np.complex128)
    piv = a[1]
    beta[1], gamma[1], delta[1] = b[1] / piv, c[1] / piv, d[1] / piv
    for i in range(2, m):
        piv = a[i] - b[i] * gamma[i - 1]
        beta[i] = -b[i] * beta[i - 1] / piv
        gamma[i] = c[i] / piv
        delta[i] = (d[i] - b[i] * delta[i - 1]) / piv
    P = 1.0 + 0.0j
    bf = df = 0.0j
    for k in range(1, m):
        bf += P * beta[k]
        df += P * delta[k]
        P = -gamma[k] * P
    gf = -P
    UA = a[0] - c[0] * bf
    UC = -c[0] * gf
    UD = d[0] - c[0] * df
    DB = -b[m] * beta[m - 1]
    DA = -b[m] * gamma[m - 1]
    DD = -b[m] * delta[m - 1]
    return UA, UC, UD, DB, DA, DD, delta[1:]


def rd_form_substitute(a, b, c, delta, psi_J, psi_K):
    """SS of the RD form: given psi_J and psi_K, the interior rows of the block follow from the
    RD rows by substitution upwards, psi_i = delta_i - beta_i psi_J - gamma_i psi_{i+1},
    i = m-1 .. 1 (beta_i, gamma_i recomputed from the matrix as in rd_form_block)."""
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    c = np.asarray(c, np.complex128)
    m = a.shape[0] - 1
    psi = np.zeros(m + 1, np.complex128)
    psi[0], psi[m] = psi_J, psi_K
    if m < 2:
        return psi
    beta = np.zeros(m, np.complex128)
    gamma = np.zeros(m, np.complex128)
    piv = a[1]
    beta[1], gamma[1] = b[1] / piv, c[1] / piv
    for i in range(2, m):
        piv = a[i] - b[i] * gamma[i - 1]
        beta[i] = -b[i] * beta[i - 1] / piv
        gamma[i] = c[i] / piv
    for i in range(m - 1, 0, -1):
        psi[i] = delta[i - 1] - beta[i] * psi_J - gamma[i] * psi[i + 1]
    return psi
