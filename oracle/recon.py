"""Accelerated forward-backward splitting (Algorithm 1, Section "Optimization").

Oracle module: test infrastructure only.

Steps, in the algorithm's order, for k = 1, 2, ...:
  select a subset Q_k of the views (given as input here, so both implementations use the same);
  d^k   = sum_{q in Q_k} Re(J_q^*(H_q(.) - y_q)) / ||y_q||^2        (gradient of the data term);
  f^k   = prox_{gamma_k tau TV + i_{>=0}}(v^k - gamma_k d^k),  gamma_k = gamma_0 / sqrt(k);
  a_{k+1} = (1 + sqrt(1 + 4 a_k^2)) / 2;
  v^{k+1} = f^k + ((a_k - 1) / a_{k+1}) (f^k - f^{k-1}),
with v^1 = f^0 and a_1 = 1.  Reading: the algorithm writes the gradient at f^k, which is only
defined on the next line; as in the accelerated method it cites, the gradient is evaluated at the
extrapolated point v^k.

``fbs`` takes the gradient and the prox as functions, so the loop itself is pinned on a problem
with a known minimiser (nonnegative least squares, tests/test_oracle_recon.py); ``reconstruct``
plugs in the Lippmann-Schwinger data term (oracle.grad) and the TV prox (oracle.tv).
"""
from __future__ import annotations

import math
from typing import Callable, List, Sequence

import numpy as np

from . import tv as _tv


def fbs(f0: np.ndarray, grad: Callable[[np.ndarray, Sequence[int]], np.ndarray],
        prox: Callable[[np.ndarray, float], np.ndarray], gamma0: float, subsets: Sequence[Sequence[int]],
        history: List | None = None) -> np.ndarray:
    """Run len(subsets) iterations; grad(v, subset) is the data-term gradient over the subset and
    prox(z, gamma) the proximity operator of gamma (tau R + i_C)."""
    f_prev = np.array(f0, dtype=np.float64)
    v = f_prev.copy()
    a = 1.0
    for k, sub in enumerate(subsets, start=1):
        gamma = gamma0 / math.sqrt(k)
        d = grad(v, sub)
        f = prox(v - gamma * d, gamma)
        a_next = (1.0 + math.sqrt(1.0 + 4.0 * a * a)) / 2.0
        v = f + ((a - 1.0) / a_next) * (f - f_prev)
        f_prev, a = f, a_next
        if history is not None:
            history.append(f.copy())
    return f_prev


def reconstruct(problem, dirs, yhat, f0, tau: float, gamma0: float, subsets, tv_iters: int,
                nonneg: bool = True, history: List | None = None) -> np.ndarray:
    """Algorithm 1 with the data term of eq. (prob) (oracle.grad.Problem) and the TV prox."""
    dirs = np.asarray(dirs)

    def grad(v, sub):
        sub = list(sub)
        _, d = problem.loss_grad(v, dirs[sub], [yhat[q] for q in sub])
        return d

    def prox(z, gamma):
        return _tv.fgp_prox(z, gamma * tau, tv_iters, nonneg)

    return fbs(f0, grad, prox, gamma0, subsets, history)
