"""Plane-wave incident fields (Section "Physical Model"; illuminations on a cone, Fig. 1).

Oracle module: test infrastructure only.

u_in(x) = exp(j k d . x), with x the signed voxel position i - n/2 + 1 along each axis and
d a unit vector; arrays are indexed [z, y, x].  Pinned by tests/test_oracle_solver.py
(phase at the origin voxel, unit modulus, and exact Helmholtz plane-wave structure).
"""
from __future__ import annotations

import numpy as np


def plane_wave(n: int, k: float, d) -> np.ndarray:
    c = np.arange(n, dtype=np.float64) - n // 2 + 1
    dx, dy, dz = (float(t) for t in d)
    phase = k * (dz * c[:, None, None] + dy * c[None, :, None] + dx * c[None, None, :])
    return np.exp(1j * phase)
