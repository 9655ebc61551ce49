"""Samples of ghat_t and the reduced-memory kernel of Proposition 2.

Oracle module: test infrastructure only.

Grids (Theorem 1): Omega_M = [[-M/2+1, M/2]]^3.  Arrays use the NumPy FFT ordering: array
index j in [0, M) stands for the signed index j if j <= M/2 else j - M, which is exactly the
element of Omega_M congruent to j mod M.  F is the unnormalised DFT with exp(-2 j pi k q / M),
F^{-1} carries 1/M per axis (numpy.fft.fftn / ifftn).

  ghat_grid(n, p, k)[q] = ghat_t(delta |q|),  q in Omega_{np},  delta = 2 pi / (n p)   (Theorem 1)

Proposition 2 defines the modified kernel on Omega_{2n}:
  gm[k] = (8/p^3) sum_{s in [[0, p/2-1]]^3} F^{-1}_{2n}( ghat_t[(p/2) . - s] )[k] exp(-2 j pi k.s / (n p))
where k is the signed index in Omega_{2n} (the phase is not 2n-periodic, so the signed
representative matters).  Substituting q = (p/2) q' - s in the inverse DFT on Omega_{np} shows
that this is the restriction of F^{-1}_{np}(ghat_grid) to Omega_{2n}; ``gm_direct`` computes it
that way and ``gm_coset`` computes the coset sum as printed.  Their agreement is an exact identity
(tests/test_oracle_kernel.py).  The volume operator uses ghat_m = F_{2n}(gm).
"""
from __future__ import annotations

import numpy as np

from . import dft, green


def signed(M: int) -> np.ndarray:
    """Signed index in Omega_M for each array index 0..M-1."""
    j = np.arange(M)
    return np.where(j <= M // 2, j, j - M)


def _radius3(a, b, c):
    return np.sqrt(a[:, None, None] ** 2 + b[None, :, None] ** 2 + c[None, None, :] ** 2)


def ghat_grid(n: int, p: int, k: float) -> np.ndarray:
    """ghat_t(delta |q|) for q in Omega_{np} (NumPy ordering), delta = 2 pi / (n p), R = sqrt(3) n."""
    M = n * p
    delta = 2.0 * np.pi / M
    q = signed(M).astype(np.float64)
    s = delta * _radius3(q, q, q)
    return green.ghat_t(s, k, np.sqrt(3.0) * n)


def gm_direct(n: int, p: int, k: float) -> np.ndarray:
    """Restriction of F^{-1}_{np}(ghat_grid) to Omega_{2n}, returned as a 2n-periodic array."""
    M = n * p
    full = dft.ifftn(ghat_grid(n, p, k))
    idx = signed(2 * n) % M          # position of each signed k in Omega_{2n} inside the np grid
    return full[np.ix_(idx, idx, idx)]


def gm_coset(n: int, p: int, k: float) -> np.ndarray:
    """Proposition 2: coset sum on the 2n grid only."""
    if p % 2 or p < 2:
        raise ValueError("p must be even and >= 2")
    M2 = 2 * n
    half = p // 2
    delta = 2.0 * np.pi / (n * p)
    R = np.sqrt(3.0) * n
    qp = signed(M2).astype(np.float64)
    kk = signed(M2).astype(np.float64)
    acc = np.zeros((M2, M2, M2), dtype=np.complex128)
    for s1 in range(half):
        for s2 in range(half):
            for s3 in range(half):
                a = half * qp - s1
                b = half * qp - s2
                c = half * qp - s3
                vals = green.ghat_t(delta * _radius3(a, b, c), k, R)
                inv = dft.ifftn(vals)
                ph1 = np.exp(-2j * np.pi * kk * s1 / (n * p))
                ph2 = np.exp(-2j * np.pi * kk * s2 / (n * p))
                ph3 = np.exp(-2j * np.pi * kk * s3 / (n * p))
                acc += inv * ph1[:, None, None] * ph2[None, :, None] * ph3[None, None, :]
    return acc * (8.0 / p ** 3)


def ghat_m(n: int, p: int, k: float, method: str = "coset") -> np.ndarray:
    """F_{2n}(gm): the Fourier-domain kernel the volume operator multiplies by."""
    gm = gm_coset(n, p, k) if method == "coset" else gm_direct(n, p, k)
    return dft.fftn(gm)
