"""Python front end of the C ABI (include/cntri.h) over torch device tensors.

Argument marshalling only: pointers, sizes and the current HIP stream go to libcntri.so,
whose kernels do every step of the solve.  PyTorch provides device memory and streams.

Names follow the paper (arXiv 2205.00856, Sec. 4, Eq. (5)): a = diagonal, b = sub-diagonal,
c = super-diagonal, d = right-hand side; psi is the wave function of the CN step (Sec. 2).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import CnLayout, CnOperator, check

__all__ = ["Layout", "Handle", "handle", "solve", "solve_noalloc", "solve_adjoint", "assemble", "rhs", "step",
           "propagate", "step_adjoint", "get_status", "describe_plan", "reserve", "autotune",
           "profile", "profile_report", "tune_cache", "radial_step",
           "propagate_adjoint", "propagate_adjoint_reconstruct"]


@dataclass
class Layout:
    """Shape of the batch (see cn_layout in include/cntri.h).

    Uniform batch: system s, row i at element s*batch_stride + i*elem_stride.
    Uneven batch: offsets (host, batch+1 values) of systems packed back to back.
    """

    n: int = 0
    batch: int = 1
    elem_stride: int = 1
    batch_stride: int = 0
    offsets: Optional[Sequence[int]] = None
    partition: int = 0
    rows_per_thread: int = 0
    shared_coefficients: bool = False  # uniform batch: all systems use system 0's a, b, c / V, x
    levels: int = 0  # partition levels before a serial RS stage (0 = automatic nesting)
    _offs_np: Optional[np.ndarray] = field(default=None, repr=False)

    @staticmethod
    def contiguous(n: int, batch: int = 1, **kw) -> "Layout":
        return Layout(n=n, batch=batch, elem_stride=1, batch_stride=n, **kw)

    @staticmethod
    def interleaved(n: int, batch: int, **kw) -> "Layout":
        return Layout(n=n, batch=batch, elem_stride=batch, batch_stride=1, **kw)

    @staticmethod
    def uneven(offsets, **kw) -> "Layout":
        offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        return Layout(n=0, batch=int(offs.shape[0] - 1), offsets=offs, _offs_np=offs, **kw)

    def rows(self) -> int:
        if self.offsets is not None:
            return int(self._np_offsets()[-1])
        return self.n * self.batch

    def span(self) -> int:
        if self.offsets is not None:
            return int(self._np_offsets()[-1])
        return (self.batch - 1) * self.batch_stride + (self.n - 1) * self.elem_stride + 1

    def _np_offsets(self) -> np.ndarray:
        if self._offs_np is None:
            self._offs_np = np.ascontiguousarray(np.asarray(self.offsets, dtype=np.int64))
        return self._offs_np

    def c(self) -> CnLayout:
        L = CnLayout()
        L.n = int(self.n)
        L.batch = int(self.batch)
        L.elem_stride = int(self.elem_stride)
        L.batch_stride = int(self.batch_stride if self.batch_stride else self.n)
        if self.offsets is not None:
            o = self._np_offsets()
            L.offsets = o.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        else:
            L.offsets = None
        L.partition = int(self.partition)
        L.rows_per_thread = int(self.rows_per_thread)
        L.shared_coefficients = 1 if self.shared_coefficients else 0
        L.levels = int(self.levels)
        return L

    def coef_span(self) -> int:
        """Elements the coefficient arrays (a, b, c / V, xgrid) must hold."""
        if self.shared_coefficients and self.offsets is None:
            return (self.n - 1) * self.elem_stride + 1
        return self.span()


class Handle:
    """Owns a cn_handle_t (workspace, plans, status flag) on one device."""

    def __init__(self, device: int = 0):
        self.device = device
        self._h = ctypes.c_void_p()
        check(_lib.lib().cn_create(ctypes.byref(self._h), device), "cn_create")

    def close(self):
        if self._h:
            _lib.lib().cn_destroy(self._h)
            self._h = ctypes.c_void_p()

    @property
    def ptr(self):
        return self._h


_handles: dict = {}


def handle(device: Optional[int] = None) -> Handle:
    if device is None:
        device = torch.cuda.current_device()
    h = _handles.get(device)
    if h is None:
        h = _handles[device] = Handle(device)
    return h


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, dtype, name: str, min_elems: int):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (strides are given by the layout)")
    if t.numel() < min_elems:
        raise ValueError(f"{name} has {t.numel()} elements, the layout needs {min_elems}")


def _layout_for(t: torch.Tensor, layout: Optional[Layout]) -> Layout:
    if layout is not None:
        return layout
    if t.dim() == 1:
        return Layout.contiguous(t.shape[0], 1)
    if t.dim() == 2:
        return Layout.contiguous(t.shape[1], t.shape[0])
    raise ValueError("give a Layout for tensors of more than two dimensions")


def _operator(V, dx, dt, xgrid=None, v_scale=1.0, dx_per_system=None, W=None) -> CnOperator:
    op = CnOperator()
    op.absorb = None if W is None else W.data_ptr()
    op.V = V.data_ptr()
    op.v_scale = float(v_scale)
    op.dx = float(dx)
    op.dx_per_system = None if dx_per_system is None else dx_per_system.data_ptr()
    op.dt = float(dt)
    op.xgrid = None if xgrid is None else xgrid.data_ptr()
    return op


def _check_op(L: Layout, V, xgrid, dx_per_system, W=None):
    span = L.coef_span()
    _need(V, torch.float64, "V", span)
    if W is not None:
        _need(W, torch.float64, "W", span)
    if xgrid is not None:
        _need(xgrid, torch.float64, "xgrid", span)
    if dx_per_system is not None:
        _need(dx_per_system, torch.float64, "dx_per_system", L.batch)


def reserve(layout: Layout, device=None):
    h = handle(device)
    Lc = layout.c()
    check(_lib.lib().cn_reserve(h.ptr, ctypes.byref(Lc)), "cn_reserve")


def describe_plan(layout: Layout, cn_mode: bool = False, device=None,
                  absorbing: bool = False) -> str:
    """The plan of cn_tridiag_solve, of the Crank-Nicolson steps (cn_mode) or of the fused
    steps with an absorbing potential (absorbing)."""
    h = handle(device)
    Lc = layout.c()
    buf = ctypes.create_string_buffer(4096)
    mode = 2 if absorbing else int(bool(cn_mode))
    check(_lib.lib().cn_describe_plan(h.ptr, ctypes.byref(Lc), mode, buf, 4096),
          "cn_describe_plan")
    return buf.value.decode()


def solve(a, b, c, d, out=None, layout: Optional[Layout] = None):
    """x = T^{-1} d (cn_tridiag_solve).  out may be d (in place)."""
    L = _layout_for(d, layout)
    span = L.span()
    for t, nm in ((a, "a"), (b, "b"), (c, "c")):
        _need(t, torch.complex128, nm, L.coef_span())
    _need(d, torch.complex128, "d", span)
    if out is None:
        out = torch.empty_like(d)
    _need(out, torch.complex128, "out", span)
    h = handle(d.device.index)
    Lc = L.c()
    check(_lib.lib().cn_tridiag_solve(h.ptr, ctypes.byref(Lc), _ptr(a), _ptr(b), _ptr(c), _ptr(d),
                                      _ptr(out), _stream(d)), "cn_tridiag_solve")
    return out


def solve_noalloc(a, b, c, d, out, layout: Optional[Layout] = None):
    """x = T^{-1} d through cn_tridiag_solve_noalloc: the library allocates no device memory
    (its fixed scratch array holds the plan's tables and workspace); out is required."""
    L = _layout_for(d, layout)
    span = L.span()
    for t, nm in ((a, "a"), (b, "b"), (c, "c")):
        _need(t, torch.complex128, nm, L.coef_span())
    _need(d, torch.complex128, "d", span)
    _need(out, torch.complex128, "out", span)
    h = handle(d.device.index)
    Lc = L.c()
    check(_lib.lib().cn_tridiag_solve_noalloc(h.ptr, ctypes.byref(Lc), _ptr(a), _ptr(b), _ptr(c),
                                              _ptr(d), _ptr(out), _stream(d)),
          "cn_tridiag_solve_noalloc")
    return out


def solve_adjoint(a, b, c, x, gx, need_abc=True, layout: Optional[Layout] = None):
    """Reverse mode of solve: returns (gd, ga, gb, gc) (ga/gb/gc None unless need_abc)."""
    L = _layout_for(x, layout)
    span = L.span()
    for t, nm in ((a, "a"), (b, "b"), (c, "c"), (x, "x"), (gx, "gx")):
        _need(t, torch.complex128, nm, span)
    gd = torch.empty_like(x)
    ga = gb = gc = None
    if need_abc:
        ga, gb, gc = torch.empty_like(x), torch.empty_like(x), torch.empty_like(x)
    h = handle(x.device.index)
    Lc = L.c()
    check(_lib.lib().cn_tridiag_solve_adjoint(h.ptr, ctypes.byref(Lc), _ptr(a), _ptr(b), _ptr(c),
                                              _ptr(x), _ptr(gx), _ptr(gd), _ptr(ga), _ptr(gb),
                                              _ptr(gc), _stream(x)), "cn_tridiag_solve_adjoint")
    return gd, ga, gb, gc


def assemble(V, dx, dt, E=0.0, xgrid=None, v_scale=1.0, dx_per_system=None,
             layout: Optional[Layout] = None, W=None):
    """Materialised coefficients (a, b, c) of T = 1 + i dt/2 H (cn_assemble)."""
    L = _layout_for(V, layout)
    _check_op(L, V, xgrid, dx_per_system, W)
    shape = V.shape
    a = torch.empty(shape, dtype=torch.complex128, device=V.device)
    b = torch.empty_like(a)
    c = torch.empty_like(a)
    op = _operator(V, dx, dt, xgrid, v_scale, dx_per_system, W)
    h = handle(V.device.index)
    Lc = L.c()
    check(_lib.lib().cn_assemble(h.ptr, ctypes.byref(Lc), ctypes.byref(op), float(E), _ptr(a),
                                 _ptr(b), _ptr(c), _stream(V)), "cn_assemble")
    return a, b, c


def rhs(psi, V, dx, dt, E=0.0, xgrid=None, v_scale=1.0, dx_per_system=None,
        layout: Optional[Layout] = None, W=None, out=None):
    """Materialised explicit half-step d = (1 - i dt/2 H) psi (cn_rhs), into out if given."""
    L = _layout_for(psi, layout)
    _need(psi, torch.complex128, "psi", L.span())
    _check_op(L, V, xgrid, dx_per_system, W)
    d = torch.empty_like(psi) if out is None else out
    _need(d, torch.complex128, "out", L.span())
    op = _operator(V, dx, dt, xgrid, v_scale, dx_per_system, W)
    h = handle(psi.device.index)
    Lc = L.c()
    check(_lib.lib().cn_rhs(h.ptr, ctypes.byref(Lc), ctypes.byref(op), float(E), _ptr(psi),
                            _ptr(d), _stream(psi)), "cn_rhs")
    return d


def step(psi, V, dx, dt, E=0.0, xgrid=None, v_scale=1.0, dx_per_system=None, out=None,
         layout: Optional[Layout] = None, W=None):
    """One Crank-Nicolson step (cn_step).  out may be psi (in place).  W: absorbing potential
    (the potential is V - iW), taken in materialised form."""
    L = _layout_for(psi, layout)
    _need(psi, torch.complex128, "psi", L.span())
    _check_op(L, V, xgrid, dx_per_system, W)
    if out is None:
        out = torch.empty_like(psi)
    _need(out, torch.complex128, "out", L.span())
    op = _operator(V, dx, dt, xgrid, v_scale, dx_per_system, W)
    h = handle(psi.device.index)
    Lc = L.c()
    check(_lib.lib().cn_step(h.ptr, ctypes.byref(Lc), ctypes.byref(op), float(E), _ptr(psi),
                             _ptr(out), _stream(psi)), "cn_step")
    return out


def propagate(psi, V, dx, dt, nsteps, E=None, xgrid=None, v_scale=1.0, dx_per_system=None,
              ckpt=None, K=1, layout: Optional[Layout] = None, W=None):
    """nsteps CN steps in place on psi (cn_propagate); E: host sequence of nsteps values."""
    L = _layout_for(psi, layout)
    _need(psi, torch.complex128, "psi", L.span())
    _check_op(L, V, xgrid, dx_per_system, W)
    Earr = None
    if E is not None:
        Earr = np.ascontiguousarray(np.asarray(E, dtype=np.float64))
        if Earr.shape[0] < nsteps:
            raise ValueError("E needs one value per step")
    if ckpt is not None:
        _need(ckpt, torch.complex128, "ckpt", ((nsteps + K - 1) // K) * L.span())
    op = _operator(V, dx, dt, xgrid, v_scale, dx_per_system, W)
    h = handle(psi.device.index)
    Lc = L.c()
    Ep = None if Earr is None else Earr.ctypes.data_as(ctypes.c_void_p)
    check(_lib.lib().cn_propagate(h.ptr, ctypes.byref(Lc), ctypes.byref(op), int(nsteps), Ep,
                                  _ptr(psi), _ptr(ckpt), int(K), _stream(psi)), "cn_propagate")
    return psi


def propagate_resident(psi, V, dx, dt, nsteps, E=None, xgrid=None, v_scale=1.0,
                       layout: Optional[Layout] = None, W=None, ckpt=None, K=1):
    """nsteps CN steps of one system in place on psi in ONE launch (cn_propagate_resident).
    Raises CnError(CN_ERR_UNSUPPORTED) for layouts or operators it does not take (then
    propagate is the call); get_status raises CnError(CN_ERR_WAIT_TIMEOUT) after a launch whose
    workgroups could not all run at once.  W: absorbing potential (the potential is V - iW);
    ckpt, K: checkpoints as in propagate."""
    L = _layout_for(psi, layout)
    _need(psi, torch.complex128, "psi", L.span())
    _check_op(L, V, xgrid, None, W)
    Earr = None
    if E is not None:
        Earr = np.ascontiguousarray(np.asarray(E, dtype=np.float64))
        if Earr.shape[0] < nsteps:
            raise ValueError("E needs one value per step")
    if ckpt is not None:
        _need(ckpt, torch.complex128, "ckpt", ((nsteps + K - 1) // K) * L.span())
    op = _operator(V, dx, dt, xgrid, v_scale, None, W)
    h = handle(psi.device.index)
    Lc = L.c()
    Ep = None if Earr is None else Earr.ctypes.data_as(ctypes.c_void_p)
    check(_lib.lib().cn_propagate_resident(h.ptr, ctypes.byref(Lc), ctypes.byref(op),
                                           int(nsteps), Ep, _ptr(psi), _ptr(ckpt), int(K),
                                           _stream(psi)),
          "cn_propagate_resident")
    return psi


def propagate_adjoint(ckpt, g, V, dx, dt, nsteps, K, E=None, xgrid=None, v_scale=1.0, dV=None,
                      dE=None, seg=None, layout: Optional[Layout] = None, W=None):
    """Reverse mode of propagate from its checkpoints (cn_propagate_adjoint).  g (in: gradient at
    psi_T, out: gradient at psi_0) is updated in place; dV (float64) accumulates; dE (float64,
    nsteps) is written when given (needs xgrid).  W: the absorbing potential of the forward."""
    L = _layout_for(g, layout)
    span = L.span()
    _need(g, torch.complex128, "g", span)
    _need(ckpt, torch.complex128, "ckpt", ((nsteps + K - 1) // K) * span)
    _check_op(L, V, xgrid, None, W)
    if seg is None:
        seg = torch.empty((K + 1) * span, dtype=torch.complex128, device=g.device)
    _need(seg, torch.complex128, "seg", (K + 1) * span)
    Earr = None
    if E is not None:
        Earr = np.ascontiguousarray(np.asarray(E, dtype=np.float64))
        if Earr.shape[0] < nsteps:
            raise ValueError("E needs one value per step")
    if dE is not None:
        _need(dE, torch.float64, "dE", nsteps)
    op = _operator(V, dx, dt, xgrid, v_scale, None, W)
    h = handle(g.device.index)
    Lc = L.c()
    Ep = None if Earr is None else Earr.ctypes.data_as(ctypes.c_void_p)
    check(_lib.lib().cn_propagate_adjoint(h.ptr, ctypes.byref(Lc), ctypes.byref(op), int(nsteps),
                                          Ep, _ptr(ckpt), int(K), _ptr(seg), _ptr(g), _ptr(dV),
                                          _ptr(dE), _stream(g)), "cn_propagate_adjoint")
    return g


def propagate_adjoint_reconstruct(psi_T, g, V, dx, dt, nsteps, K, E=None, xgrid=None,
                                  v_scale=1.0, dV=None, dE=None, seg=None,
                                  layout: Optional[Layout] = None, W=None):
    """Reverse mode of propagate without checkpoints (cn_propagate_adjoint_reconstruct): the
    states are rebuilt backwards from the final state psi_T (read only) segment by segment of K
    steps.  g, dV, dE as in propagate_adjoint.  Real potentials only: with W the library
    refuses (CN_ERR_UNSUPPORTED)."""
    L = _layout_for(g, layout)
    span = L.span()
    _need(g, torch.complex128, "g", span)
    _need(psi_T, torch.complex128, "psi_T", span)
    _check_op(L, V, xgrid, None, W)
    m = min(K, nsteps)
    if seg is None:
        seg = torch.empty((m + 1) * span, dtype=torch.complex128, device=g.device)
    _need(seg, torch.complex128, "seg", (m + 1) * span)
    Earr = None
    if E is not None:
        Earr = np.ascontiguousarray(np.asarray(E, dtype=np.float64))
        if Earr.shape[0] < nsteps:
            raise ValueError("E needs one value per step")
    if dE is not None:
        _need(dE, torch.float64, "dE", nsteps)
    op = _operator(V, dx, dt, xgrid, v_scale, None, W)
    h = handle(g.device.index)
    Lc = L.c()
    Ep = None if Earr is None else Earr.ctypes.data_as(ctypes.c_void_p)
    check(_lib.lib().cn_propagate_adjoint_reconstruct(
        h.ptr, ctypes.byref(Lc), ctypes.byref(op), int(nsteps), Ep, _ptr(psi_T), int(K),
        _ptr(seg), _ptr(g), _ptr(dV), _ptr(dE), _stream(g)), "cn_propagate_adjoint_reconstruct")
    return g


def step_adjoint(psi_n, psi_np1, g_np1, V, dx, dt, E=0.0, xgrid=None, v_scale=1.0, dV=None,
                 dE_out=None, g_out=None, layout: Optional[Layout] = None, W=None):
    """One step of the adjoint recursion (cn_step_adjoint).  Returns g_n; accumulates into dV
    (float64, in place) and writes dE_out[0] when given (needs xgrid).  W: absorbing potential."""
    L = _layout_for(psi_n, layout)
    span = L.span()
    for t, nm in ((psi_n, "psi_n"), (psi_np1, "psi_np1"), (g_np1, "g_np1")):
        _need(t, torch.complex128, nm, span)
    _check_op(L, V, xgrid, None, W)
    if g_out is None:
        g_out = torch.empty_like(psi_n)
    op = _operator(V, dx, dt, xgrid, v_scale, None, W)
    h = handle(psi_n.device.index)
    Lc = L.c()
    check(_lib.lib().cn_step_adjoint(h.ptr, ctypes.byref(Lc), ctypes.byref(op), float(E),
                                     _ptr(psi_n), _ptr(psi_np1), _ptr(g_np1), _ptr(g_out),
                                     _ptr(dV), _ptr(dE_out), _stream(psi_n)), "cn_step_adjoint")
    return g_out


def radial_step(psi, V, dr, dt, E, l0, nl, out=None):
    """One partial-wave step (cn_radial_step): psi is l-major, nl waves of len(V) radial points
    r_j = j dr.  out may be psi (in place)."""
    nr = V.shape[0]
    _need(V, torch.float64, "V", nr)
    _need(psi, torch.complex128, "psi", nl * nr)
    if out is None:
        out = torch.empty_like(psi)
    _need(out, torch.complex128, "out", nl * nr)
    op = _lib.CnRadial()
    op.nr, op.l0, op.nl = int(nr), int(l0), int(nl)
    op.V = V.data_ptr()
    op.dr, op.dt = float(dr), float(dt)
    h = handle(psi.device.index)
    check(_lib.lib().cn_radial_step(h.ptr, ctypes.byref(op), float(E), _ptr(psi), _ptr(out),
                                    _stream(psi)), "cn_radial_step")
    return out


def tune_cache(path: Optional[str], device=None):
    """Persistent autotune cache file (cn_tune_cache); None stops using one."""
    h = handle(device)
    check(_lib.lib().cn_tune_cache(h.ptr, None if path is None else path.encode()),
          "cn_tune_cache")


def profile(enable: bool = True, device=None):
    """Plan log on/off (cn_profile): HIP events around every launch of the following calls."""
    h = handle(device)
    check(_lib.lib().cn_profile(h.ptr, 1 if enable else 0), "cn_profile")


def profile_report(device=None) -> list:
    """The logged launches since the last report (cn_profile_report): a list of
    (label, milliseconds) in launch order."""
    h = handle(device)
    buf = ctypes.create_string_buffer(1 << 20)
    check(_lib.lib().cn_profile_report(h.ptr, buf, 1 << 20), "cn_profile_report")
    out = []
    for line in buf.value.decode().splitlines():
        label, _, ms = line.rpartition(" ms=")
        out.append((label, float(ms)))
    return out


def get_status(device=None) -> int:
    """Synchronises the current stream; 1 if a non-finite result was met since the last call."""
    h = handle(device)
    dev = torch.device("cuda", h.device)
    return check(_lib.lib().cn_get_status(h.ptr, ctypes.c_void_p(
        torch.cuda.current_stream(dev).cuda_stream)), "cn_get_status")


def autotune(layout: Layout, d, x, a=None, b=None, c=None, V=None, dx=1.0, dt=0.0, E=0.0,
             xgrid=None, v_scale=1.0, dx_per_system=None, sequence: bool = False) -> str:
    """cn_autotune: time the candidate tiles on these buffers (cn_step if V is given, else
    cn_tridiag_solve; with sequence=True, 8 chained steps as cn_propagate runs them) and keep
    the fastest for later calls with this layout.  x is overwritten.  Returns the report."""
    cn_mode = (2 if sequence else 1) if V is not None else 0
    span = layout.span()
    _need(d, torch.complex128, "d/psi", span)
    _need(x, torch.complex128, "x", span)
    op = None
    if cn_mode:
        _check_op(layout, V, xgrid, dx_per_system)
        op = _operator(V, dx, dt, xgrid, v_scale, dx_per_system)
    else:
        for t, nm in ((a, "a"), (b, "b"), (c, "c")):
            _need(t, torch.complex128, nm, span)
    h = handle(d.device.index)
    Lc = layout.c()
    buf = ctypes.create_string_buffer(8192)
    check(_lib.lib().cn_autotune(h.ptr, ctypes.byref(Lc), int(cn_mode),
                                 ctypes.byref(op) if op is not None else None, float(E), _ptr(a),
                                 _ptr(b), _ptr(c), _ptr(d), _ptr(x), buf, 8192, _stream(d)),
          "cn_autotune")
    return buf.value.decode()
