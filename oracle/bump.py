"""Closed-form continuous reference for Theorem 1's accuracy statement.

Oracle module: test infrastructure only.

For a radial bump v(x) = (1 - |x|^2/a^2)^q on |x| < a, averaging g over spheres (the
Helmholtz shell theorem) gives the exact convolution with the free-space Green function:
  (g * v)(r) = int_0^a v(rho) rho (exp(j k (r + rho)) - exp(j k |r - rho|)) / (2 j k r) d rho,
  (g * v)(0) = int_0^a v(rho) rho exp(j k rho) d rho.
On Omega (support of v inside the cube) g * v = g_t * v, so the discrete G of Theorem 1 must
approach it as n and p grow (error bound of Theorem 1).  Evaluated with adaptive quadrature.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate


def bump(r, a: float, q: int):
    r = np.asarray(r, dtype=np.float64)
    return np.where(r < a, np.clip(1.0 - (r / a) ** 2, 0.0, None) ** q, 0.0)


def conv_exact(r: float, k: float, a: float, q: int) -> complex:
    v = lambda rho: (1.0 - (rho / a) ** 2) ** q
    if r == 0.0:
        fr = lambda rho: v(rho) * rho * np.cos(k * rho)
        fi = lambda rho: v(rho) * rho * np.sin(k * rho)
    else:
        def kern(rho):
            return (np.exp(1j * k * (r + rho)) - np.exp(1j * k * abs(r - rho))) / (2j * k * r)
        fr = lambda rho: v(rho) * rho * kern(rho).real
        fi = lambda rho: v(rho) * rho * kern(rho).imag
    pts = [r] if 0.0 < r < a else None
    re = integrate.quad(fr, 0.0, a, points=pts, epsabs=1e-14, epsrel=1e-13, limit=400)[0]
    im = integrate.quad(fi, 0.0, a, points=pts, epsabs=1e-14, epsrel=1e-13, limit=400)[0]
    return complex(re, im)
