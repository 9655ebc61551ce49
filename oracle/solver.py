"""Solution of the discrete Lippmann-Schwinger system (I - G diag f) u = u_in, eq. (lipp1).

Oracle module: test infrastructure only.

The paper solves this system with a Krylov method and names BiCGSTAB (van der Vorst).  The
recurrence below is the unpreconditioned van der Vorst BiCGSTAB with these readings (the paper
does not spell them out):
  * x0 = b, r0 = b - A x0, shadow residual rh = r0;  <a, b> = sum conj(a) b.
  * stop when ||r|| / ||b|| <= tol, checked on s after the first half step as well;
  * breakdown |rho| <= eps ||rh|| ||r|| or omega == 0: restart with rh = r, p = v = 0;
  * after the loop, the true residual b - A x is recomputed; if it exceeds tol and restarts
    remain, the iteration restarts from x.
The same recurrence runs on the GPU with FP64 scalars.  Pinned against a dense LU solve on
tiny grids; the restart branches by a breakdown threshold that fires, one that fires at every step
(the plain two-stage descent), and a true-residual restart equal to a fresh solve from the restart
point (tests/test_oracle_solver.py).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class SolveInfo:
    status: int = 1          # 0 converged, 1 max iterations, 2 breakdown unrecovered
    iters: int = 0
    matvecs: int = 0
    restarts: int = 0
    relres_rec: float = np.nan
    relres_true: float = np.nan
    history: list = dataclasses.field(default_factory=list)


def bicgstab(A, b: np.ndarray, tol: float, maxit: int = 500, x0=None, max_restarts: int = 3,
             eps: float = np.finfo(np.float64).eps):
    """Return (x, info).  A is a callable acting on arrays shaped like b."""
    info = SolveInfo()
    nb = np.sqrt(np.vdot(b, b).real)
    x = b.copy() if x0 is None else x0.copy()
    if nb == 0.0:
        info.status, info.relres_rec, info.relres_true = 0, 0.0, 0.0
        return np.zeros_like(b), info
    r = b - A(x)
    info.matvecs += 1
    rr = np.sqrt(np.vdot(r, r).real)
    info.relres_rec = rr / nb
    if rr / nb <= tol:
        info.status = 0
        info.relres_true = info.relres_rec
        return x, info

    def fresh(rvec):
        return rvec.copy(), np.zeros_like(rvec), np.zeros_like(rvec), 1.0 + 0j, 1.0 + 0j, 1.0 + 0j

    rh, p, v, rho_prev, alpha, omega = fresh(r)
    restarts = 0
    it = 0
    while True:
        converged = False
        while it < maxit:
            it += 1
            rho = np.vdot(rh, r)
            nrh = np.sqrt(np.vdot(rh, rh).real)
            if abs(rho) <= eps * nrh * rr:
                rh, p, v, rho_prev, alpha, omega = fresh(r)
                rho = np.vdot(rh, r)
                restarts += 1
            beta = (rho / rho_prev) * (alpha / omega)
            p = r + beta * (p - omega * v)
            v = A(p)
            info.matvecs += 1
            alpha = rho / np.vdot(rh, v)
            s = r - alpha * v
            ns = np.sqrt(np.vdot(s, s).real)
            if ns / nb <= tol:
                x = x + alpha * p
                rr = ns
                info.history.append(ns / nb)
                converged = True
                break
            t = A(s)
            info.matvecs += 1
            omega = np.vdot(t, s) / np.vdot(t, t)
            x = x + alpha * p + omega * s
            r = s - omega * t
            rho_prev = rho
            rr = np.sqrt(np.vdot(r, r).real)
            info.history.append(rr / nb)
            if rr / nb <= tol:
                converged = True
                break
            if omega == 0:
                rh, p, v, rho_prev, alpha, omega = fresh(r)
                restarts += 1
        info.relres_rec = rr / nb
        r_true = b - A(x)
        info.matvecs += 1
        rt = np.sqrt(np.vdot(r_true, r_true).real)
        info.relres_true = rt / nb
        if rt / nb <= tol:
            info.status = 0
            break
        if it >= maxit or restarts >= max_restarts:
            info.status = 1 if it >= maxit else 2
            break
        # restart from the current iterate with the true residual
        r = r_true
        rr = rt
        rh, p, v, rho_prev, alpha, omega = fresh(r)
        restarts += 1
        del converged
    info.iters = it
    info.restarts = restarts
    return x, info


def dense_solve(G: np.ndarray, f: np.ndarray, b: np.ndarray) -> np.ndarray:
    """(I - G diag f)^{-1} b with a dense LU factorisation (tiny grids only)."""
    N = b.size
    A = np.eye(N, dtype=np.complex128) - G * f.ravel()[None, :]
    return np.linalg.solve(A, b.ravel()).reshape(b.shape)
