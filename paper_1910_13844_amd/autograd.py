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


class LSDetector(torch.autograd.Function):
    """y_q = D_q P G~_m diag(f) u_q(f) on an m x m camera (eq. (lipp2) with the pupil / propagation P
    of numerical aperture `na` and defocus `dz`, and decimation by `q`).  Backward: the chain's
    adjoints (ls_decimate transpose, ls_pupil adjoint, ls_farfield_wide_adj with conjugation) give the
    volume right-hand side of the adjoint solve, ls_vjp_rhs the gradient."""

    @staticmethod
    def forward(ctx, f, lsctx: Context, dirs, m: int, na, dz: float, q: int, tol: float, maxit: int):
        fc = f.detach().contiguous()
        u, info = lsctx.ls_forward(fc, dirs, tol=tol, maxit=maxit)
        y = lsctx.ls_farfield_wide(m, fc, u)
        if na is not None:
            y = lsctx.ls_pupil(y, na, dz)
        if q > 1:
            y = lsctx.ls_decimate(y, q)
        ctx.save_for_backward(fc, u)
        ctx.lsctx, ctx.m, ctx.na, ctx.dz, ctx.q, ctx.tol, ctx.maxit = lsctx, m, na, dz, q, tol, maxit
        ctx.forward_info = info
        return y

    @staticmethod
    def backward(ctx, gy: torch.Tensor):
        f, u = ctx.saved_tensors
        c = ctx.lsctx
        h = gy.contiguous()
        if ctx.q > 1:
            h = c.ls_decimate(h, ctx.q, m=ctx.m, transpose=True)
        if ctx.na is not None:
            h = c.ls_pupil(h, ctx.na, ctx.dz, adjoint=True)
        b = c.ls_farfield_wide_adj(ctx.m, h, conj=True)
        grad, _ = c.ls_vjp_rhs(f, u, b, tol=ctx.tol, maxit=ctx.maxit)
        return grad, None, None, None, None, None, None, None, None


def detector_fields(f: torch.Tensor, lsctx: Context, dirs: Sequence, m: int, na=None, dz: float = 0.0, q: int = 1,
                    tol: float = 1e-5, maxit: int = 500) -> torch.Tensor:
    """Differentiable camera fields [Q, m/q, m/q] through the detector chain D_q P G~_m."""
    return LSDetector.apply(f, lsctx, dirs, m, na, dz, q, tol, maxit)


class DataTerm(torch.autograd.Function):
    """The data term of eq. (prob), L = sum_q ||y_q - ymeas_q||^2 / (2 ||ymeas_q||^2), computed by
    ls_residual, which also returns its gradient with respect to y, (y_q - ymeas_q) / ||ymeas_q||^2
    (PyTorch's dL/dRe(y) + i dL/dIm(y))."""

    @staticmethod
    def forward(ctx, y: torch.Tensor, y_meas: torch.Tensor, lsctx: Context):
        gy, _, loss = lsctx.ls_residual(y.detach(), y_meas, weighted=True)
        ctx.save_for_backward(gy)
        return loss

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (gy,) = ctx.saved_tensors
        return g.to(gy.real.dtype) * gy, None, None


def data_loss(y: torch.Tensor, y_meas: torch.Tensor, lsctx: Context) -> torch.Tensor:
    """sum_q ||y_q - ymeas_q||^2 / (2 ||ymeas_q||^2), the data term of eq. (prob) (a 0-dim float64
    tensor on the device), differentiable in y."""
    return DataTerm.apply(y, y_meas, lsctx)
