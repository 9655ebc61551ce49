"""Incident fields: plane waves (Section "Physical Model"; illuminations on a cone) and volumes
propagated from a measured detector field (Section "Computation of the 3D Incident Field", Fig. 3).

Oracle module: test infrastructure only.

u_in(x) = exp(j k d . x), with x the signed voxel position i - n/2 + 1 along each axis and
d a unit vector; arrays are indexed [z, y, x].  Pinned by tests/test_oracle_solver.py
(phase at the origin voxel, unit modulus, and exact Helmholtz plane-wave structure).
``angular_spectrum`` is pinned by tests/test_oracle_incident.py (plane waves reproduced exactly,
tilt transfer vs plain propagation, identity at zero distance, composition).
"""
from __future__ import annotations

import numpy as np

from . import dft


def plane_wave(n: int, k: float, d) -> np.ndarray:
    c = np.arange(n, dtype=np.float64) - n // 2 + 1
    dx, dy, dz = (float(t) for t in d)
    phase = k * (dz * c[:, None, None] + dy * c[None, :, None] + dx * c[None, None, :])
    return np.exp(1j * phase)


# ---------------------------------------------------------------------------------------------
# Incident field from a measured detector field (Section "Computation of the 3D Incident Field").
#
# The field y_in measured on the detector plane x3 = x_Gamma is propagated to each slice z of the
# volume by the angular spectrum method: in the lateral Fourier domain the propagator is
#     p_z(w) = exp(-i (x_Gamma - z) sqrt(k^2 - |w|^2)),
# read with k^2 (the printed radicand has k) and with the evanescent part |w| > k dropped (it would
# grow exponentially when propagating back from the detector; the paper does not discuss it).
# Tilt transfer: y_in = a exp(i x~.k~) with a slowly varying amplitude a; the propagation is done on
# a = y_in exp(-i x~.k~) with the propagator evaluated at w + k~, and the result is modulated back by
# exp(i x~.k~).  The detector grid is the lateral voxel grid (m = n, spacing h = 1), x~ the signed
# positions i - n/2 + 1, and the lateral convolution is periodic over that grid, as the paper does it.
# Array frequencies follow numpy.fft.fftfreq (index n/2 is -n/2).


def lateral_freqs(n: int) -> np.ndarray:
    """Angular frequency (radians per voxel) of each DFT index."""
    return 2.0 * np.pi * np.fft.fftfreq(n)


def propagator(n: int, k: float, dist: float, shift=(0.0, 0.0)) -> np.ndarray:
    """p(w + shift) over the [ky, kx] DFT grid for a propagation distance dist = x_Gamma - z."""
    w = lateral_freqs(n)
    wy = w[:, None] + shift[1]
    wx = w[None, :] + shift[0]
    s2 = k * k - (wx * wx + wy * wy)
    kz = np.sqrt(np.maximum(s2, 0.0))
    return np.where(s2 >= 0.0, np.exp(-1j * dist * kz), 0.0)


def angular_spectrum(y_in: np.ndarray, k: float, xg: float, ktilde=(0.0, 0.0), tilt_transfer: bool = True
                     ) -> np.ndarray:
    """u_in [z, y, x] on the n^3 grid from the detector field y_in [y, x] at x3 = xg."""
    n = y_in.shape[0]
    c = np.arange(n, dtype=np.float64) - n // 2 + 1
    kx, ky = (float(t) for t in ktilde) if tilt_transfer else (0.0, 0.0)
    carrier = np.exp(1j * (kx * c[None, :] + ky * c[:, None]))
    a_hat = dft.fft2(y_in * np.conj(carrier))
    out = np.empty((n, n, n), dtype=np.complex128)
    for iz in range(n):
        out[iz] = dft.ifft2(a_hat * propagator(n, k, xg - c[iz], (kx, ky))) * carrier
    return out
