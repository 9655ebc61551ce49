"""Proximity operator of gamma tau TV + i_{>=0} (Section "Optimization", prox step of Algorithm 1).

Oracle module: test infrastructure only.

The paper evaluates this prox with the fast gradient-projection method on the dual of the
total-variation problem (its reference for TV).  Readings (the paper does not spell them out):
  * TV is isotropic: TV(x) = sum_v || (Dx)_v ||_2 with forward differences
    (Dx)_v = (x_v - x_{v+e_z}, x_v - x_{v+e_y}, x_v - x_{v+e_x}), a difference that would leave the
    grid being 0 (Neumann boundary);
  * the constraint set is C = {x >= 0} (or all of R^N when nonneg is False).

Dual problem.  TV(x) = max_{p in P} <D^T p, x> over P = {p : ||p_v||_2 <= 1, p zero where the
difference leaves the grid}.  Exchanging min and max in
    min_{x in C} 1/2 ||x - b||^2 + lam TV(x)
gives, for each p, the minimiser x(p) = P_C(b - lam D^T p) and the dual value
    dual(p) = 1/2 ||b||^2 - 1/2 ||w||^2 + 1/2 ||w - P_C(w)||^2,   w = b - lam D^T p,
a concave function of p whose gradient is lam D x(p).  Fast gradient projection runs Nesterov's
accelerated projected gradient ascent on it, with step 1 / (lam L) where L = 12 bounds ||D||^2 in
three dimensions (each of the three difference operators has norm squared at most 4).

``fgp_prox`` follows those steps; ``dual_gap`` = primal(x(p)) - dual(p) >= 0 certifies a result
independently of how p was found (tests/test_oracle_recon.py).
"""
from __future__ import annotations

import numpy as np


def diff(x: np.ndarray) -> np.ndarray:
    """D x: forward differences along z, y, x, shape (3,) + x.shape; zero on the far face."""
    d = np.zeros((3,) + x.shape, dtype=x.dtype)
    d[0, :-1] = x[:-1] - x[1:]
    d[1, :, :-1] = x[:, :-1] - x[:, 1:]
    d[2, :, :, :-1] = x[:, :, :-1] - x[:, :, 1:]
    return d


def diff_T(p: np.ndarray) -> np.ndarray:
    """D^T p (the adjoint of ``diff``): <D x, p> = <x, D^T p> for every x."""
    p0, p1, p2 = p[0].copy(), p[1].copy(), p[2].copy()
    p0[-1] = 0.0
    p1[:, -1] = 0.0
    p2[:, :, -1] = 0.0
    out = p0 + p1 + p2
    out[1:] -= p0[:-1]
    out[:, 1:] -= p1[:, :-1]
    out[:, :, 1:] -= p2[:, :, :-1]
    return out


def tv(x: np.ndarray) -> float:
    """Isotropic total variation."""
    return float(np.sum(np.sqrt(np.sum(diff(x) ** 2, axis=0))))


def project_P(p: np.ndarray) -> np.ndarray:
    """Per-voxel projection onto the unit ball, with the components that leave the grid zeroed."""
    q = p.copy()
    q[0, -1] = 0.0
    q[1, :, -1] = 0.0
    q[2, :, :, -1] = 0.0
    nrm = np.sqrt(np.sum(q ** 2, axis=0))
    return q / np.maximum(1.0, nrm)


def project_C(x: np.ndarray, nonneg: bool) -> np.ndarray:
    return np.maximum(x, 0.0) if nonneg else x


def primal(x: np.ndarray, b: np.ndarray, lam: float) -> float:
    return 0.5 * float(np.sum((x - b) ** 2)) + lam * tv(x)


def dual(p: np.ndarray, b: np.ndarray, lam: float, nonneg: bool) -> float:
    w = b - lam * diff_T(p)
    return 0.5 * float(np.sum(b ** 2)) - 0.5 * float(np.sum(w ** 2)) + 0.5 * float(np.sum((w - project_C(w, nonneg)) ** 2))


def fgp_prox(b: np.ndarray, lam: float, iters: int, nonneg: bool = True, return_dual: bool = False):
    """argmin_x 1/2 ||x - b||^2 + lam TV(x) + i_C(x) by ``iters`` fast gradient-projection steps."""
    b = np.asarray(b, dtype=np.float64)
    if lam <= 0.0:
        x = project_C(b, nonneg)
        return (x, np.zeros((3,) + b.shape)) if return_dual else x
    p_prev = np.zeros((3,) + b.shape)
    r = p_prev.copy()
    t = 1.0
    for _ in range(iters):
        # ascent step on the dual at r, then projection onto P
        x_r = project_C(b - lam * diff_T(r), nonneg)
        p = project_P(r + diff(x_r) / (12.0 * lam))
        t_next = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        r = p + ((t - 1.0) / t_next) * (p - p_prev)
        p_prev, t = p, t_next
    x = project_C(b - lam * diff_T(p_prev), nonneg)
    return (x, p_prev) if return_dual else x


def dual_gap(b: np.ndarray, lam: float, p: np.ndarray, nonneg: bool = True) -> float:
    """primal(x(p)) - dual(p) for the dual point p (>= 0; zero only at the solution)."""
    x = project_C(b - lam * diff_T(p), nonneg)
    return primal(x, b, lam) - dual(p, b, lam, nonneg)
