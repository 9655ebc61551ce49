"""The discrete volume operator G of Theorem 1 / Proposition 2, four ways.

Oracle module: test infrastructure only.

Vectors v live on Omega_n = [[-n/2+1, n/2]]^3; array index i in [0, n) holds the signed
position i - n/2 + 1 (so x = 0 sits at i = n/2 - 1).  Arrays are indexed [z, y, x].

  G_fft       Proposition 2:  (G v)[k] = F^{-1}_{2n}( ghat_m . F_{2n}(v_2) )[k],  k in Omega_n,
              v_2 = v zero-extended to Omega_{2n} at its signed positions.
  G_theorem1  Theorem 1:      same with the p-fold zero padding and ghat_t sampled on Omega_{np}.
  G_direct    the plain discrete convolution  (G v)[k] = sum_{k' in Omega_n} gm[k - k'] v[k'].
  G_dense     the N x N matrix G[k, k'] = gm[k - k'].

The first two agree exactly (Proposition 2), and both agree with the last two because a
circular convolution of size >= 2n has no wrap-around on Omega_n (differences of two points of
Omega_n lie in [[-(n-1), n-1]]).  These identities are tested in tests/test_oracle_ops.py.
"""
from __future__ import annotations

import numpy as np

from . import dft
from . import kernel as _kernel


def _embed(v: np.ndarray, M: int) -> np.ndarray:
    """Place v (n^3, signed positions of Omega_n) into an M^3 periodic grid."""
    n = v.shape[0]
    idx = (np.arange(n) - n // 2 + 1) % M
    out = np.zeros((M, M, M), dtype=np.complex128)
    out[np.ix_(idx, idx, idx)] = v
    return out


def _crop(w: np.ndarray, n: int) -> np.ndarray:
    M = w.shape[0]
    idx = (np.arange(n) - n // 2 + 1) % M
    return w[np.ix_(idx, idx, idx)]


def G_fft(ghat_m: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Proposition 2 form on the 2n grid."""
    n = v.shape[0]
    assert ghat_m.shape == (2 * n,) * 3
    w = dft.ifftn(ghat_m * dft.fftn(_embed(v, 2 * n)))
    return _crop(w, n)


def G_theorem1(n: int, p: int, k: float, v: np.ndarray) -> np.ndarray:
    """Theorem 1 form on the np grid."""
    gt = _kernel.ghat_grid(n, p, k)
    w = dft.ifftn(gt * dft.fftn(_embed(v, n * p)))
    return _crop(w, n)


def G_direct(gm: np.ndarray, v: np.ndarray) -> np.ndarray:
    """O(N^2) discrete convolution with the 2n-periodic kernel gm (signed differences)."""
    n = v.shape[0]
    M = gm.shape[0]
    pos = np.arange(n)
    out = np.zeros((n, n, n), dtype=np.complex128)
    for z in range(n):
        for y in range(n):
            dz = (z - pos) % M
            dy = (y - pos) % M
            for x in range(n):
                dx = (x - pos) % M
                out[z, y, x] = np.sum(gm[np.ix_(dz, dy, dx)] * v)
    return out


def G_point(gm: np.ndarray, v: np.ndarray, z: int, y: int, x: int) -> complex:
    """One output of the direct sum (used to sample large grids)."""
    n = v.shape[0]
    M = gm.shape[0]
    pos = np.arange(n)
    return complex(np.sum(gm[np.ix_((z - pos) % M, (y - pos) % M, (x - pos) % M)] * v))


def G_dense(gm: np.ndarray, n: int) -> np.ndarray:
    """Dense matrix of G on Omega_n, row/column order = C order of [z, y, x]."""
    M = gm.shape[0]
    pos = np.arange(n)
    Z, Y, X = np.meshgrid(pos, pos, pos, indexing="ij")
    Z, Y, X = Z.ravel(), Y.ravel(), X.ravel()
    return gm[(Z[:, None] - Z[None, :]) % M, (Y[:, None] - Y[None, :]) % M, (X[:, None] - X[None, :]) % M]


def A_apply(ghat_m: np.ndarray, f: np.ndarray, x: np.ndarray) -> np.ndarray:
    """A x = x - G (f . x): the Lippmann-Schwinger operator of eq. (lipp1)."""
    return x - G_fft(ghat_m, f * x)
