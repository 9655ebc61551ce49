"""torch.autograd.Function over the forward model y_q(f) = G~ diag(f) u_q(f), eqs. (lipp1)-(lipp2).

Forward runs ls_forward (BiCGSTAB for every illumination) and ls_farfield; backward runs ls_vjp,
the Jacobian-adjoint product of Algorithm 1's gradient step (one more solve per illumination).
PyTorch passes gy = dL/dRe(y) + i dL/dIm(y) for a real loss L; ls_vjp returns Re(J^* gy), the
gradient with respect to the real potential f.
"""
from __future__ import annotations

from typing import Sequence

import torch

from .api import Context


class LSFarField(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f: torch.Tensor, lsctx: Context, dirs, tol: float, maxit: int):
        fc = f.detach().contiguous()
        u, info = lsctx.ls_forward(fc, dirs, tol=tol, maxit=maxit)
        y = lsctx.ls_farfield(fc, u)
        ctx.save_for_backward(fc, u)
        ctx.lsctx = lsctx
        ctx.tol, ctx.maxit = tol, maxit
        ctx.forward_info = info
        return y

    @staticmethod
    def backward(ctx, gy: torch.Tensor):
        f, u = ctx.saved_tensors
        grad, _ = ctx.lsctx.ls_vjp(f, u, gy.contiguous(), tol=ctx.tol, maxit=ctx.maxit)
        return grad, None, None, None, None


def farfield(f: torch.Tensor, lsctx: Context, dirs: Sequence, tol: float = 1e-5, maxit: int = 500) -> torch.Tensor:
    """Differentiable detector fields y [Q, n, n] for potential f [n, n, n] and plane waves `dirs`."""
    return LSFarField.apply(f, lsctx, dirs, tol, maxit)


def data_loss(y: torch.Tensor, y_meas: torch.Tensor) -> torch.Tensor:
    """sum_q ||y_q - ymeas_q||^2 / (2 ||ymeas_q||^2), the data term of eq. (prob)."""
    r = (y - y_meas).reshape(y.shape[0], -1)
    m = y_meas.reshape(y.shape[0], -1)
    return (r.abs() ** 2).sum(dim=1).div(2.0 * (m.abs() ** 2).sum(dim=1)).sum()
