"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module only draws numbers: grids, potentials, wave functions, random systems.  It holds
none of the method's arithmetic (no coefficient assembly, no right-hand side, no solve), so
that the oracle and the HIP path stay independent.

Workloads (shapes and distributions of the paper's TDSE use case, Sec. 2-3; the paper itself
measures only a 3e5-point 1D box whose potential it does not state):

  plain_1d        N=65536, dx=0.1, dt=0.02, soft-core V, Gaussian psi0 (sigma 5, k0 1)
  adi_2d          4096 x 4096 grid, dx=dy=0.1, dt=0.01, 2D soft-core V, random psi0
  large_system    N=2^28 explicit system: V_j ~ U(-1,0) on dx=0.01, dt=0.02; d ~ CN(0,1)
  uneven_batch    10000 systems, lengths log-uniform in [256, 65536], own dx ~ U(0.05,0.2)
  differentiated  N=2^20, dx=0.05, dt=0.01, 2000 steps, field E_k ~ N(0, 0.05^2)

All draws use numpy's PCG64 generator; the order of draws is fixed per workload.
"""
from __future__ import annotations

import hashlib

import numpy as np

SEED_BASE = 1000


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def grid_1d(n: int, dx: float) -> np.ndarray:
    """x_j = (j - (n+1)/2) dx for j = 1..n (x centred on 0, walls at j = 0 and n+1)."""
    j = np.arange(1, n + 1, dtype=np.float64)
    return (j - (n + 1) / 2.0) * dx


def softcore(x: np.ndarray, soft: float = 2.0) -> np.ndarray:
    return -1.0 / np.sqrt(x * x + soft)


def gaussian(x: np.ndarray, x0: float, sigma: float, k0: float, dx: float) -> np.ndarray:
    """exp(-(x-x0)^2/(2 sigma^2) + i k0 x), normalised so that sum |psi|^2 dx = 1."""
    psi = np.exp(-((x - x0) ** 2) / (2.0 * sigma * sigma) + 1j * k0 * x)
    return psi / np.sqrt(np.sum(np.abs(psi) ** 2) * dx)


def complex_normal(g: np.random.Generator, shape) -> np.ndarray:
    """Re, Im ~ N(0, 1) independently (real parts drawn first, then imaginary parts)."""
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    return re + 1j * im


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


# ----------------------------------------------------------------------------- workloads
def plain_1d(n: int = 65536, dx: float = 0.1, dt: float = 0.02, steps: int = 200):
    x = grid_1d(n, dx)
    return dict(name="plain_1d", n=n, dx=dx, dt=dt, steps=steps, x=x, V=softcore(x),
                psi0=gaussian(x, 0.0, 5.0, 1.0, dx))


def absorber(n: int, frac: float = 0.1, strength: float = 2.0) -> np.ndarray:
    """A quadratic absorbing ramp W >= 0 over the outer `frac` of the box at both walls, zero
    inside: the usual shape of a complex absorbing potential (the potential is V - iW)."""
    j = np.arange(n, dtype=np.float64)
    width = max(1.0, frac * n)
    depth = np.maximum(0.0, np.maximum(width - j, j - (n - 1 - width)) / width)
    return strength * depth * depth


def absorbing_1d(n: int = 65536, dx: float = 0.1, dt: float = 0.02, steps: int = 200):
    """The plain 1D workload with an absorbing ramp over the outer tenth of the box, and the
    wave packet started inside the right ramp (at 93 % of the box), moving toward the wall."""
    x = grid_1d(n, dx)
    return dict(name="absorbing_1d", n=n, dx=dx, dt=dt, steps=steps, x=x, V=softcore(x),
                W=absorber(n), psi0=gaussian(x, x[int(0.93 * n)], 5.0, 2.0, dx))


def adi_2d(n: int = 4096, dx: float = 0.1, dt: float = 0.01, steps: int = 100,
           seed: int = SEED_BASE + 1):
    g = rng(seed)
    x = grid_1d(n, dx)
    y = grid_1d(n, dx)
    X, Y = np.meshgrid(x, y)  # (ny, nx), x fastest
    V = -1.0 / np.sqrt(X * X + Y * Y + 2.0)
    psi = complex_normal(g, (n, n))
    psi /= np.sqrt(np.sum(np.abs(psi) ** 2) * dx * dx)
    return dict(name="adi_2d", nx=n, ny=n, dx=dx, dy=dx, dt=dt, steps=steps, V=V, psi0=psi)


def large_system(n: int = 1 << 28, dx: float = 0.01, dt: float = 0.02,
                 seed: int = SEED_BASE + 2):
    """V_j ~ U(-1, 0), then d_j with Re, Im ~ N(0, 1)."""
    g = rng(seed)
    V = g.uniform(-1.0, 0.0, n)
    d = complex_normal(g, n)
    return dict(name="large_system", n=n, dx=dx, dt=dt, V=V, d=d)


def uneven_lengths(g: np.random.Generator, batch: int, lo: int = 256, hi: int = 65536):
    u = g.uniform(0.0, 1.0, batch)
    return np.rint(lo * (hi / lo) ** u).astype(np.int64)


def uneven_batch(batch: int = 10000, lo: int = 256, hi: int = 65536, dt: float = 0.02,
                 steps: int = 50, seed: int = SEED_BASE + 3):
    """Lengths log-uniform in [lo, hi]; dx_s ~ U(0.05, 0.2); V ~ U(-2, 0); psi ~ CN(0,1)
    normalised per system (sum |psi|^2 dx_s = 1).  Systems are packed back to back."""
    g = rng(seed)
    lengths = uneven_lengths(g, batch, lo, hi)
    dxs = g.uniform(0.05, 0.2, batch)
    offsets = np.zeros(batch + 1, np.int64)
    np.cumsum(lengths, out=offsets[1:])
    total = int(offsets[-1])
    V = g.uniform(-2.0, 0.0, total)
    psi = complex_normal(g, total)
    for s in range(batch):
        o0, o1 = offsets[s], offsets[s + 1]
        psi[o0:o1] /= np.sqrt(np.sum(np.abs(psi[o0:o1]) ** 2) * dxs[s])
    return dict(name="uneven_batch", batch=batch, offsets=offsets, lengths=lengths, dx=dxs,
                dt=dt, steps=steps, V=V, psi0=psi)


def differentiated(n: int = 1 << 20, dx: float = 0.05, dt: float = 0.01, steps: int = 2000,
                   ckpt: int = 50, seed: int = SEED_BASE + 4):
    """Soft-core V plus a length-gauge field x E_k with E ~ N(0, 0.05^2); psi0 the plain_1d
    Gaussian; target phi_T a Gaussian whose centre ~ U(15, 25), width ~ U(4, 7) and
    momentum ~ U(0.8, 1.2) are drawn from the seed (after E)."""
    g = rng(seed)
    x = grid_1d(n, dx)
    E = g.normal(0.0, 0.05, steps)
    c0 = g.uniform(15.0, 25.0)
    sg = g.uniform(4.0, 7.0)
    k = g.uniform(0.8, 1.2)
    return dict(name="differentiated", n=n, dx=dx, dt=dt, steps=steps, ckpt=ckpt, x=x,
                V=softcore(x), E=E, psi0=gaussian(x, 0.0, 5.0, 1.0, dx),
                phi=gaussian(x, c0, sg, k, dx), phi_params=(c0, sg, k))


# ----------------------------------------------------------------------- random systems
def random_system(n: int, seed: int, kind: str = "dd"):
    """Random tridiagonal test systems (a, b, c, d), complex128.

    kind "dd":   |a_i| >= |b_i| + |c_i| + 1 (strictly diagonally dominant)
    kind "herm": Hermitian part positive definite: a = 1 + u + i v, b, c = i * real
                 symmetric off-diagonals (the class every CN matrix with real V belongs to)
    """
    g = rng(seed)
    if kind == "dd":
        b = complex_normal(g, n)
        c = complex_normal(g, n)
        ph = g.uniform(0.0, 2 * np.pi, n)
        mag = np.abs(b) + np.abs(c) + 1.0 + g.uniform(0.0, 1.0, n)
        a = mag * np.exp(1j * ph)
    elif kind == "herm":
        off = g.standard_normal(n)
        b = 1j * off
        c = 1j * np.roll(off, -1)
        a = 1.0 + g.uniform(0.0, 1.0, n) + 1j * g.standard_normal(n) * 3.0
    else:
        raise ValueError(kind)
    d = complex_normal(g, n)
    return a, b, c, d


def random_cn(n: int, seed: int, dx: float = 0.1, dt: float = 0.02, vlo: float = -2.0,
              vhi: float = 0.0):
    """Random potential and wave function for a CN step on n points."""
    g = rng(seed)
    V = g.uniform(vlo, vhi, n)
    psi = complex_normal(g, n)
    return dict(n=n, dx=dx, dt=dt, V=V, psi=psi)
