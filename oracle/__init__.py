"""CPU oracle for the Crank-Nicolson tridiagonal path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import this package.  The product library (``paper_2205_00856_amd``) never imports,
links or calls it, and the two share no code.

What it computes (arXiv 2205.00856):

* ``thomas``            -- x = T^{-1} d by serial elimination without pivoting: the RS stage of
                           Table 1 applied to the whole system (Sec. 2 last paragraph, Sec. 4.1.5).
* ``cn_coeffs``/``cn_rhs``/``cn_step``/``cn_propagate`` -- the CN step of Sec. 2, Eqs. (2)-(4),
                           with the three-point Laplacian and Dirichlet walls.  ``W`` adds an
                           absorbing potential (V - iW); the step is then the Cayley form
                           (1 + i tau H)^{-1} (1 - i tau H), whose right side is not T^dagger.
* ``adi_step``          -- one Lie-split ADI step (operator splitting, Sec. 3) on a 2D grid.
* ``radial_step``       -- one Lie-split partial-wave step (Sec. 3): CN in r per l with the
                           centrifugal term, then CN in l per r with the field coupling.
* ``thomas_adjoint``    -- reverse mode of the solve (plain definition, lambda = T^{-H} G).
* ``cn_propagate_grad`` -- reverse mode of many CN steps with every state stored (with ``W``,
                           of the absorbing step: lambda = T^{-H} G, G_k = B^H lambda with
                           B = 1 - i tau H no longer equal to T^H).

Everything runs in FP64 / complex128 in the C file ``cn_oracle.c`` (built with gcc -O2
-ffp-contract=off, OpenMP only across independent systems).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cn_oracle.c")
_LIB = os.path.join(_HERE, "libcn_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    d = ctypes.c_double
    ci = ctypes.c_int
    lib.oracle_thomas.argtypes = [i64, P, P, P, P, P, P]
    lib.oracle_thomas_batched.argtypes = [i64, P, P, P, P, P, P, ci]
    lib.oracle_cn_coeffs.argtypes = [i64, P, d, d, P, d, P, P, P]
    lib.oracle_cn_coeffs.restype = None
    lib.oracle_cn_rhs.argtypes = [i64, P, P, d, d, P, d, P]
    lib.oracle_cn_rhs.restype = None
    lib.oracle_cn_step.argtypes = [i64, P, d, d, P, d, P, P]
    lib.oracle_cn_propagate.argtypes = [i64, P, d, d, i64, P, P, P]
    lib.oracle_cn_coeffs_w.argtypes = [i64, P, d, d, P, d, P, P, P, P]
    lib.oracle_cn_coeffs_w.restype = None
    lib.oracle_cn_rhs_w.argtypes = [i64, P, P, d, d, P, d, P, P]
    lib.oracle_cn_rhs_w.restype = None
    lib.oracle_cn_step_w.argtypes = [i64, P, d, d, P, d, P, P, P]
    lib.oracle_cn_propagate_w.argtypes = [i64, P, d, d, i64, P, P, P, P]
    lib.oracle_cn_step_batched.argtypes = [i64, P, P, P, d, P, P, ci]
    lib.oracle_adi_step.argtypes = [i64, i64, P, d, d, d, P, ci]
    lib.oracle_thomas_adjoint.argtypes = [i64, P, P, P, P, P, P, P, P, P]
    lib.oracle_cn_propagate_grad.argtypes = [i64, P, d, d, i64, P, P, P, P, P, P, P]
    lib.oracle_cn_propagate_grad_w.argtypes = [i64, P, d, d, i64, P, P, P, P, P, P, P, P]
    lib.oracle_radial_step.argtypes = [i64, i64, i64, P, d, d, d, P]
    lib.oracle_max_threads.argtypes = []
    _lib = lib
    return lib


def _c(x, dtype):
    return np.ascontiguousarray(x, dtype=dtype)


def _p(x):
    return None if x is None else x.ctypes.data_as(ctypes.c_void_p)


class OracleBreakdown(RuntimeError):
    pass


def _check(st):
    if st != 0:
        raise OracleBreakdown("zero or non-finite pivot in the oracle elimination")


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def thomas(a, b, c, d):
    """x = T^{-1} d for one system (b[0], c[-1] ignored)."""
    lib = _load()
    a, b, c, d = (_c(v, np.complex128) for v in (a, b, c, d))
    n = a.shape[0]
    x = np.empty(n, np.complex128)
    w = np.empty(2 * max(n, 1), np.complex128)
    _check(lib.oracle_thomas(n, _p(a), _p(b), _p(c), _p(d), _p(x), _p(w)))
    return x


def thomas_batched(offsets, a, b, c, d, nthreads: int = 0):
    """Packed systems, system s = rows offsets[s]:offsets[s+1]."""
    lib = _load()
    offsets = _c(offsets, np.int64)
    a, b, c, d = (_c(v, np.complex128) for v in (a, b, c, d))
    x = np.empty_like(d)
    _check(lib.oracle_thomas_batched(offsets.shape[0] - 1, _p(offsets), _p(a), _p(b), _p(c),
                                     _p(d), _p(x), nthreads))
    return x


def cn_coeffs(V, dx, dt, xgrid=None, E=0.0, W=None):
    """T = 1 + i tau H; with W the potential is V - iW (absorbing, non-Hermitian H)."""
    lib = _load()
    V = _c(V, np.float64)
    xg = None if xgrid is None else _c(xgrid, np.float64)
    Wa = None if W is None else _c(W, np.float64)
    n = V.shape[0]
    a, b, c = (np.empty(n, np.complex128) for _ in range(3))
    lib.oracle_cn_coeffs_w(n, _p(V), dx, dt, _p(xg), E, _p(Wa), _p(a), _p(b), _p(c))
    return a, b, c


def cn_rhs(psi, V, dx, dt, xgrid=None, E=0.0, W=None):
    """d = (1 - i tau H) psi (Sec. 2, Eq. (3)); with W the potential is V - iW."""
    lib = _load()
    psi = _c(psi, np.complex128)
    V = _c(V, np.float64)
    xg = None if xgrid is None else _c(xgrid, np.float64)
    Wa = None if W is None else _c(W, np.float64)
    d = np.empty_like(psi)
    lib.oracle_cn_rhs_w(psi.shape[0], _p(psi), _p(V), dx, dt, _p(xg), E, _p(Wa), _p(d))
    return d


def cn_step(psi, V, dx, dt, xgrid=None, E=0.0, W=None):
    lib = _load()
    psi = _c(psi, np.complex128)
    V = _c(V, np.float64)
    xg = None if xgrid is None else _c(xgrid, np.float64)
    Wa = None if W is None else _c(W, np.float64)
    out = np.empty_like(psi)
    _check(lib.oracle_cn_step_w(psi.shape[0], _p(V), dx, dt, _p(xg), E, _p(Wa), _p(psi),
                                _p(out)))
    return out


def cn_propagate(psi, V, dx, dt, nsteps, xgrid=None, E=None, W=None):
    lib = _load()
    psi = _c(psi, np.complex128).copy()
    V = _c(V, np.float64)
    xg = None if xgrid is None else _c(xgrid, np.float64)
    Ea = None if E is None else _c(E, np.float64)
    Wa = None if W is None else _c(W, np.float64)
    _check(lib.oracle_cn_propagate_w(psi.shape[0], _p(V), dx, dt, int(nsteps), _p(xg), _p(Ea),
                                     _p(Wa), _p(psi)))
    return psi


def cn_step_batched(offsets, psi, V, dx, dt, nthreads: int = 0):
    lib = _load()
    offsets = _c(offsets, np.int64)
    psi = _c(psi, np.complex128)
    V = _c(V, np.float64)
    dx = _c(dx, np.float64)
    out = np.empty_like(psi)
    _check(lib.oracle_cn_step_batched(offsets.shape[0] - 1, _p(offsets), _p(V), _p(dx), dt,
                                      _p(psi), _p(out), nthreads))
    return out


def adi_step(psi2d, V2d, dx, dy, dt, nthreads: int = 0):
    """One Lie-split ADI step; psi2d is (ny, nx) row-major with x fastest."""
    lib = _load()
    psi = _c(psi2d, np.complex128).copy()
    V = _c(V2d, np.float64)
    ny, nx = psi.shape
    _check(lib.oracle_adi_step(nx, ny, _p(V), dx, dy, dt, _p(psi), nthreads))
    return psi


def thomas_adjoint(a, b, c, x, G):
    lib = _load()
    a, b, c, x, G = (_c(v, np.complex128) for v in (a, b, c, x, G))
    n = a.shape[0]
    lam, ga, gb, gc = (np.empty(n, np.complex128) for _ in range(4))
    _check(lib.oracle_thomas_adjoint(n, _p(a), _p(b), _p(c), _p(x), _p(G), _p(lam), _p(ga),
                                     _p(gb), _p(gc)))
    return lam, ga, gb, gc


def cn_propagate_grad(psi0, V, dx, dt, nsteps, G_T, xgrid=None, E=None, W=None):
    """Returns (grad psi0, dL/dV, dL/dE or None); with W the potential is V - iW."""
    lib = _load()
    psi0 = _c(psi0, np.complex128)
    G_T = _c(G_T, np.complex128)
    V = _c(V, np.float64)
    xg = None if xgrid is None else _c(xgrid, np.float64)
    Ea = None if E is None else _c(E, np.float64)
    Wa = None if W is None else _c(W, np.float64)
    n = psi0.shape[0]
    gpsi0 = np.empty(n, np.complex128)
    dV = np.empty(n, np.float64)
    dE = np.empty(int(nsteps), np.float64) if Ea is not None else None
    _check(lib.oracle_cn_propagate_grad_w(n, _p(V), dx, dt, int(nsteps), _p(xg), _p(Ea), _p(Wa),
                                          _p(psi0), _p(G_T), _p(gpsi0), _p(dV), _p(dE)))
    return gpsi0, dV, dE


def radial_step(psi, V, dr, dt, E, l0, nl):
    """One partial-wave step; psi is l-major (nl x nr), V has nr values (r_j = j dr)."""
    lib = _load()
    psi = _c(psi, np.complex128).copy()
    V = _c(V, np.float64)
    nr = V.shape[0]
    assert psi.shape[0] == nl * nr
    _check(lib.oracle_radial_step(nr, int(l0), int(nl), _p(V), dr, dt, E, _p(psi)))
    return psi
