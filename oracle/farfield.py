"""The detector operator G~ of eq. (lipp2) (Section "Green's Function Discretization for the
Measurements").

Oracle module: test infrastructure only.

The paper writes the field on the plane x3 = x_Gamma as a sum over z-slices (rectangle rule
along z, weight h) of 2D aperiodic convolutions with the free-space Green function, evaluated
"in the same way as Theorem 1" with detector sampling equal to the volume sampling.  It gives
no formula for the lateral kernel.  Reading used here (and on the GPU): the rectangle rule is
applied laterally as well, with the untruncated g of eq. (def:Green) sampled on the voxel grid:

  y[a] = sum_{k3 in Omega_n} sum_{b in Omega_n^2} g( (a - b), x_Gamma - k3 ) v[k3, b],   a in Omega_m^2

in voxel units (the h^3 of the quadrature is absorbed by f~ = f h^2 and g(hX) = g~(X)/h),
with v = f . u, m = n and detector pixel a at the same lateral positions as the voxels.
x_Gamma > n/2 keeps g away from its singularity.  ``farfield_direct`` is that double sum
written out; ``farfield_fft`` evaluates each slice's 2D linear convolution with 2n-padded FFTs
(the fast form of the paper, O(n M log M)); their agreement is exact up to rounding
(tests/test_oracle_farfield.py).  ``farfield_T`` is the transpose G~^T used by the gradient.
"""
from __future__ import annotations

import numpy as np

from . import dft, green


def _signed_n(n):
    return np.arange(n, dtype=np.float64) - n // 2 + 1


def slice_kernels(n: int, k: float, xg: float) -> np.ndarray:
    """Spatial lateral kernels g(d, x_Gamma - k3) on the 2n-periodic offset grid, one per slice.

    Shape (n, 2n, 2n): [slice z][dy][dx] with offsets in Omega_{2n} (NumPy order).
    """
    M = 2 * n
    j = np.arange(M)
    d = np.where(j <= n, j, j - M).astype(np.float64)
    k3 = _signed_n(n)
    out = np.empty((n, M, M), dtype=np.complex128)
    for iz in range(n):
        Z = xg - k3[iz]
        r = np.sqrt(d[:, None] ** 2 + d[None, :] ** 2 + Z * Z)
        out[iz] = green.g_free(r, k)
    return out


def farfield_direct(v: np.ndarray, k: float, xg: float) -> np.ndarray:
    """Brute-force O(M N) double sum; v indexed [z, y, x]; returns [y, x] on the detector."""
    n = v.shape[0]
    c = _signed_n(n)
    out = np.zeros((n, n), dtype=np.complex128)
    for iz in range(n):
        Z = xg - c[iz]
        for ay in range(n):
            dy = c[ay] - c
            for ax in range(n):
                dx = c[ax] - c
                r = np.sqrt(dy[:, None] ** 2 + dx[None, :] ** 2 + Z * Z)
                out[ay, ax] += np.sum(green.g_free(r, k) * v[iz])
    return out


def _pad2(a, M):
    n = a.shape[-1]
    out = np.zeros(a.shape[:-2] + (M, M), dtype=np.complex128)
    out[..., :n, :n] = a
    return out


def farfield_fft(v: np.ndarray, k: float, xg: float, kern=None) -> np.ndarray:
    """Sum over slices of 2n-padded FFT linear convolutions (corner placement, then crop)."""
    n = v.shape[0]
    M = 2 * n
    if kern is None:
        kern = slice_kernels(n, k, xg)
    Kh = dft.fft2(kern)
    Vh = dft.fft2(_pad2(v, M))
    Y = dft.ifft2(np.sum(Kh * Vh, axis=0))
    return Y[:n, :n]


def farfield_T(r: np.ndarray, k: float, xg: float, kern=None) -> np.ndarray:
    """Transpose G~^T: (G~^T r)[k3, b] = sum_a g(a - b, x_Gamma - k3) r[a]  (no conjugation)."""
    n = r.shape[0]
    M = 2 * n
    if kern is None:
        kern = slice_kernels(n, k, xg)
    Kh = dft.fft2(kern)
    Rh = dft.fft2(_pad2(r, M))
    # correlation with an even kernel equals convolution
    out = dft.ifft2(Kh * Rh[None])
    return out[:, :n, :n]


def farfield_T_direct(r: np.ndarray, k: float, xg: float) -> np.ndarray:
    """Brute-force transpose, for tiny grids."""
    n = r.shape[0]
    c = _signed_n(n)
    out = np.zeros((n, n, n), dtype=np.complex128)
    for iz in range(n):
        Z = xg - c[iz]
        for by in range(n):
            dy = c - c[by]
            for bx in range(n):
                dx = c - c[bx]
                rr = np.sqrt(dy[:, None] ** 2 + dx[None, :] ** 2 + Z * Z)
                out[iz, by, bx] = np.sum(green.g_free(rr, k) * r)
    return out
