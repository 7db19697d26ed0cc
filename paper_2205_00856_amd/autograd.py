"""Autograd wrappers over the C ABI (reverse mode runs in the library's adjoint kernels).

CNSolve      x = T^{-1} d for a tridiagonal T (a, b, c, d complex128); backward solves the
             conjugate-transposed system with the same N-shaped method (cn_tridiag_solve_adjoint).
CNPropagate  psi_T after nsteps Crank-Nicolson steps with H_k = H_0 + diag(V + x E_k) (Sec. 2);
             backward (cn_propagate_adjoint) recomputes each segment of K steps forward from a
             stored checkpoint and runs the adjoint recursion backwards through it; with
             reconstruct=True no checkpoint is stored and the backward rebuilds the segments
             backwards from psi_T (cn_propagate_adjoint_reconstruct).

Complex gradients use torch's convention (d/dRe + i d/dIm of a real loss), for which
  grad d = T^{-H} grad x,  grad a_i = -lambda_i conj(x_i),  grad b_i = -lambda_i conj(x_{i-1}),
  grad c_i = -lambda_i conj(x_{i+1}),
and for the CN step psi_{k+1} = T_k^{-1} (1 - i tau H_k) psi_k (tau = dt/2, real potential):
  lambda_k = T_k^{-H} G_{k+1},  G_k = T_k lambda_k,
  dL/dV_j += tau Im(conj(lambda_k,j)(psi_k,j + psi_k+1,j)),  dL/dE_k = sum_j x_j (same term).
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import api

__all__ = ["CNSolve", "CNPropagate", "cn_solve", "cn_propagate"]


class CNSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, b, c, d, layout: Optional[api.Layout] = None):
        x = api.solve(a, b, c, d, layout=layout)
        ctx.save_for_backward(a, b, c, x)
        ctx.layout = layout
        return x

    @staticmethod
    def backward(ctx, gx):
        a, b, c, x = ctx.saved_tensors
        need = ctx.needs_input_grad
        gd, ga, gb, gc = api.solve_adjoint(a, b, c, x, gx.contiguous(),
                                           need_abc=any(need[:3]), layout=ctx.layout)
        return (ga if need[0] else None, gb if need[1] else None, gc if need[2] else None,
                gd if need[3] else None, None)


def cn_solve(a, b, c, d, layout: Optional[api.Layout] = None):
    return CNSolve.apply(a, b, c, d, layout)


class CNPropagate(torch.autograd.Function):
    """Checkpointed propagation.  E (nsteps field values) and V are float64 tensors; the
    field enters through xgrid (float64, same length as psi) when given.  W (float64, or None)
    is an absorbing potential, V - iW (constant: it receives no gradient)."""

    @staticmethod
    def forward(ctx, psi0, V, E, dx: float, dt: float, xgrid, K: int, v_scale: float = 1.0,
                W=None, reconstruct: bool = False, resident: bool = False):
        nsteps = int(E.shape[0]) if E is not None else 0
        if nsteps < 1:
            raise ValueError("CNPropagate needs at least one step (E has one value per step)")
        if reconstruct and W is not None:
            raise ValueError("reconstruct needs a real potential (the inverse step with W amplifies)")
        Eh = E.detach().cpu().numpy().astype(np.float64) if E.is_cuda else \
            E.detach().numpy().astype(np.float64)
        L = api.Layout.contiguous(psi0.shape[0], 1)
        nseg = (nsteps + K - 1) // K
        ckpt = None if reconstruct else torch.empty(nseg * psi0.shape[0], dtype=psi0.dtype,
                                                    device=psi0.device)
        psi = psi0.detach().clone()
        if resident:
            # all steps in one launch (the GPU to itself; layouts it does not take raise)
            api.propagate_resident(psi, V.detach(), dx, dt, nsteps, E=Eh, xgrid=xgrid,
                                   v_scale=v_scale, layout=L, W=W, ckpt=ckpt, K=K)
        else:
            api.propagate(psi, V.detach(), dx, dt, nsteps, E=Eh, xgrid=xgrid, v_scale=v_scale,
                          ckpt=ckpt, K=K, layout=L, W=W)
        ctx.W = W
        ctx.reconstruct = reconstruct
        # the checkpoints, or (reconstruct) the final state the backward rebuilds from
        ctx.save_for_backward(V, xgrid if xgrid is not None else torch.empty(0),
                              psi.clone() if reconstruct else ckpt)
        ctx.meta = (Eh, dx, dt, K, v_scale, nsteps, xgrid is not None, E.device, E.dtype)
        return psi

    @staticmethod
    def backward(ctx, gT):
        V, xg, ckpt = ctx.saved_tensors
        Eh, dx, dt, K, v_scale, nsteps, has_x, Edev, Edt = ctx.meta
        xgrid = xg if has_x else None
        n = gT.shape[0]
        dev = gT.device
        dV = torch.zeros(n, dtype=torch.float64, device=dev)
        dE = torch.zeros(nsteps, dtype=torch.float64, device=dev) if has_x else None
        g = gT.contiguous().clone()
        if ctx.reconstruct:
            api.propagate_adjoint_reconstruct(ckpt, g, V.detach(), dx, dt, nsteps, K, E=Eh,
                                              xgrid=xgrid, v_scale=v_scale, dV=dV, dE=dE)
        else:
            api.propagate_adjoint(ckpt, g, V.detach(), dx, dt, nsteps, K, E=Eh, xgrid=xgrid,
                                  v_scale=v_scale, dV=dV, dE=dE, W=ctx.W)
        gE = dE.to(device=Edev, dtype=Edt) if has_x else None
        return g, dV, gE, None, None, None, None, None, None, None, None


def cn_propagate(psi0, V, E, dx, dt, xgrid=None, K=50, v_scale=1.0, W=None,
                 reconstruct: bool = False, resident: bool = False):
    """resident: the forward runs as one resident launch (cn_propagate_resident) instead of the
    chained passes; the reverse mode is the same."""
    return CNPropagate.apply(psi0, V, E, dx, dt, xgrid, K, v_scale, W, reconstruct, resident)
