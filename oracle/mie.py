"""Scattering of a scalar plane wave by a homogeneous penetrable sphere (Mie series).

Oracle module: test infrastructure only.  Used as the physics reference the paper compares
against in its bead experiment (Fig. 2, "Analytical solution").  The paper prints no numbers
for that comparison, so agreement of the discrete solution with this series is a physics-level
check (its tolerance is derived in the tests from the discretisation, not from the paper):
parity of the HIP path is always taken against ``solver``/``ops``, never against this module.

Incident field exp(j k z) (time convention exp(-j w t), outgoing h_l = j_l + j y_l, matching
the Green function of eq. (def:Green)).  With k1 = k eta_s / eta_b inside r < a:
  outside  u = exp(j k z) + sum_l (2l+1) j^l A_l h_l(k r) P_l(cos t)
  inside   u =              sum_l (2l+1) j^l B_l j_l(k1 r) P_l(cos t)
A_l, B_l from continuity of u and du/dr at r = a (solved as a 2x2 system per l).
Self-check (tests/test_oracle_mie.py): both boundary conditions hold to 1e-12 at r = a, and the
series for eta_s = eta_b reduces to the incident wave.
"""
from __future__ import annotations

import numpy as np
from scipy import special as sp


def _h(l, x, derivative=False):
    return sp.spherical_jn(l, x, derivative) + 1j * sp.spherical_yn(l, x, derivative)


def coefficients(k: float, k1: float, a: float, lmax: int):
    A = np.zeros(lmax + 1, dtype=np.complex128)
    B = np.zeros(lmax + 1, dtype=np.complex128)
    for l in range(lmax + 1):
        M = np.array([[_h(l, k * a), -sp.spherical_jn(l, k1 * a)],
                      [k * _h(l, k * a, True), -k1 * sp.spherical_jn(l, k1 * a, True)]], dtype=np.complex128)
        rhs = -np.array([sp.spherical_jn(l, k * a), k * sp.spherical_jn(l, k * a, True)], dtype=np.complex128)
        A[l], B[l] = np.linalg.solve(M, rhs)
    return A, B


def default_lmax(k: float, k1: float, a: float) -> int:
    x = max(k, k1) * a
    return int(np.ceil(x + 4.0 * x ** (1.0 / 3.0) + 10))


def total_field_points(k: float, eta_ratio: float, a: float, pts: np.ndarray, lmax: int | None = None):
    """Total field at points (P, 3) given as (x, y, z) coordinates, sphere centred at 0."""
    k1 = k * eta_ratio
    if lmax is None:
        lmax = default_lmax(k, k1, a)
    A, B = coefficients(k, k1, a, lmax)
    x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]
    r = np.sqrt(x * x + y * y + z * z)
    ct = np.where(r > 0, z / np.where(r > 0, r, 1.0), 1.0)
    out = np.zeros(r.shape, dtype=np.complex128)
    inside = r < a
    for l in range(lmax + 1):
        Pl = sp.eval_legendre(l, ct)
        c = (2 * l + 1) * (1j ** l)
        out[inside] += c * B[l] * sp.spherical_jn(l, k1 * r[inside]) * Pl[inside]
        ro = r[~inside]
        out[~inside] += c * A[l] * _h(l, k * ro) * Pl[~inside]
    out[~inside] += np.exp(1j * k * z[~inside])
    return out


def total_field_grid(n: int, k: float, eta_ratio: float, a: float):
    """Total field on the voxel grid of Omega_n, indexed [z, y, x]."""
    c = np.arange(n, dtype=np.float64) - n // 2 + 1
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return total_field_points(k, eta_ratio, a, pts).reshape(n, n, n)
