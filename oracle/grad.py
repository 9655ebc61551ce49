"""Data-fidelity term and its gradient (Section "Problem Formulation", eq. (prob); Algorithm 1,
gradient step; Section "Optimization", Jacobian paragraph).

Oracle module: test infrastructure only.

  H_q(f) = G~ diag(f) u_q,   u_q = (I - G diag f)^{-1} u_in,q       eqs. (lipp1)-(lipp2), P = I
  loss   = sum_q ||H_q(f) - yhat_q||^2 / (2 ||yhat_q||^2)
  d      = sum_q Re( J_q^* (H_q(f) - yhat_q) ) / ||yhat_q||^2

Differentiating eq. (lipp1) gives J_q = G~ (I - diag(f) G)^{-1} diag(u_q).  The adjoint needs
one more solve, with (I - G^* diag f) -- the paper's printed operator mixes G~ into it, read
here as G.  Because G is complex symmetric (its kernel is even), (I - G^* D)^{-1} z =
conj((I - G D)^{-1} conj z), so
  Re(J^* r) = Re(u . w),   w = (I - G diag f)^{-1} G~^T conj(r),
a forward-type solve on conjugated data.  ``grad_adjoint`` implements that;
``grad_explicit`` builds J^* with the conjugated dense operator (tiny grids) and is the
independent check, together with central finite differences and the dot-product test
<J df, r>_R = <df, Re J^* r> (tests/test_oracle_grad.py).

``vjp`` is the same map for an arbitrary upstream gradient gy = dL/dRe(y) + j dL/dIm(y):
it returns Re(J^* gy), the gradient of L with respect to the real potential.
"""
from __future__ import annotations

import numpy as np

from . import farfield, incident, ops, solver


class Problem:
    """Forward model for one potential f on an n^3 grid, with cached kernels."""

    def __init__(self, ghat_m, n, k, xg, tol=1e-12, maxit=1000):
        self.ghat_m = ghat_m
        self.n = n
        self.k = k
        self.xg = xg
        self.tol = tol
        self.maxit = maxit
        self.kern = farfield.slice_kernels(n, k, xg)

    def A(self, f):
        return lambda x: ops.A_apply(self.ghat_m, f, x)

    def total_field(self, f, d):
        b = incident.plane_wave(self.n, self.k, d)
        u, info = solver.bicgstab(self.A(f), b, self.tol, self.maxit)
        return u, info

    def H(self, f, u):
        return farfield.farfield_fft(f * u, self.k, self.xg, self.kern)

    def forward(self, f, dirs):
        us, ys = [], []
        for d in dirs:
            u, _ = self.total_field(f, d)
            us.append(u)
            ys.append(self.H(f, u))
        return np.array(us), np.array(ys)

    def vjp(self, f, us, gys):
        """Re(J^* gy) summed over views, via the conjugated forward solve."""
        g = np.zeros(f.shape, dtype=np.float64)
        for u, gy in zip(us, gys):
            b = farfield.farfield_T(np.conj(gy), self.k, self.xg, self.kern)
            w, _ = solver.bicgstab(self.A(f), b, self.tol, self.maxit)
            g += np.real(u * w)
        return g

    def loss_grad(self, f, dirs, yhat):
        us, ys = self.forward(f, dirs)
        loss = 0.0
        gys = []
        for y, yh in zip(ys, yhat):
            nyh = np.vdot(yh, yh).real
            r = y - yh
            loss += np.vdot(r, r).real / (2.0 * nyh)
            gys.append(r / nyh)
        return loss, self.vjp(f, us, gys)

    def loss(self, f, dirs, yhat):
        _, ys = self.forward(f, dirs)
        return sum(np.vdot(y - yh, y - yh).real / (2.0 * np.vdot(yh, yh).real) for y, yh in zip(ys, yhat))


def grad_explicit(Gd, f, us, rs, weights, k, xg):
    """sum_q w_q Re(J_q^H r_q) with J^H = diag(conj u) (I - G^H diag f)^{-1} G~^H, all dense.

    Uses the conjugate transpose of the assembled matrices and the brute-force G~^T; it does
    not use the symmetry of G, so it is independent of the conjugation identity behind
    ``Problem.vjp`` (tiny grids only).
    """
    n = f.shape[0]
    N = n ** 3
    AH = np.eye(N, dtype=np.complex128) - np.conj(Gd).T * f.ravel()[None, :]
    g = np.zeros(N)
    for u, r, wq in zip(us, rs, weights):
        GtH_r = np.conj(farfield.farfield_T_direct(np.conj(r), k, xg)).ravel()
        w = np.linalg.solve(AH, GtH_r)
        g += wq * np.real(np.conj(u.ravel()) * w)
    return g.reshape(f.shape)
