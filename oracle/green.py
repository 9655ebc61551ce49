"""Fourier transform of the truncated Green function (Section "Green's Function
Discretization for the Volume", eqs. (GreenL) and (GreenL2)).

Oracle module: test infrastructure only.

Definitions (voxel units):
  g(x)   = exp(j k |x|) / (4 pi |x|)                       eq. (def:Green)
  g_t(x) = rect(|x| / (2 R')) g(x), truncated at radius R = sqrt(3) L
  ghat_t(w) = int g_t(x) exp(-j w.x) dx                     forward FT convention of the appendix

For a radial function the 3D FT reduces to a 1D integral (s = |w|):
  ghat_t(s) = (4 pi / s) int_0^R r g(r) sin(s r) dr = (1/s) int_0^R exp(j k r) sin(s r) dr.
Writing sin(sr) = (exp(jsr) - exp(-jsr)) / (2j) and E(a) = int_0^R exp(j a r) dr
              = R exp(j a R / 2) sinc(a R / 2),   sinc(x) = sin(x)/x,
gives the closed form used here, with no removable singularity anywhere:
  ghat_t(s) = (E(k + s) - E(k - s)) / (2 j s)      (s > 0)
  ghat_t(0) = int_0^R r exp(j k r) dr = (exp(j k R)(1 - j k R) - 1) / k^2.

Reading of the paper: the printed eq. (GreenL) has "+ j k sqrt3 L sinc(...)" inside the
bracket.  With "+" its numerator does not vanish at |w| = k_b, so eq. (GreenL2) could not be
its continuous extension; with "-" it equals the closed form above (and GreenL2 follows by
L'Hopital).  ``ghat_t_printed(sign=-1)`` is that corrected formula and is tested against
``ghat_t``; ``sign=+1`` is the printed one, kept to show it disagrees with direct quadrature.

Pins (tests/test_oracle_green.py): 1D adaptive quadrature of the radial integral at random s;
eq. (GreenL2) at s = k; the s = 0 limit; the corrected eq. (GreenL) away from s = k.
"""
from __future__ import annotations

import numpy as np


def _sinc(x):
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    nz = x != 0.0
    out[nz] = np.sin(x[nz]) / x[nz]
    return out


def _E(a, R):
    """E(a) = int_0^R exp(j a r) dr."""
    a = np.asarray(a, dtype=np.float64)
    return R * np.exp(0.5j * a * R) * _sinc(0.5 * a * R)


def ghat_t(s, k: float, R: float):
    """Fourier transform of g truncated at radius R, evaluated at radial frequency s >= 0."""
    s = np.asarray(s, dtype=np.float64)
    out = np.empty(s.shape, dtype=np.complex128)
    pos = s > 0.0
    sp = s[pos]
    out[pos] = (_E(k + sp, R) - _E(k - sp, R)) / (2j * sp)
    out[~pos] = (np.exp(1j * k * R) * (1.0 - 1j * k * R) - 1.0) / (k * k)
    return out


def ghat_t_printed(s, k: float, R: float, sign: int = -1):
    """Eq. (GreenL) as printed (sign=+1) or with the sinc sign corrected (sign=-1).

    1/(s^2 - k^2) * (1 - e^{jkR} (cos(R s) + sign * j k R sinc(R s))), valid for s != k.
    """
    s = np.asarray(s, dtype=np.float64)
    return (1.0 - np.exp(1j * k * R) * (np.cos(R * s) + sign * 1j * k * R * _sinc(R * s))) / (s * s - k * k)


def ghat_t_at_k(k: float, R: float):
    """Eq. (GreenL2): the value on the sphere |w| = k_b."""
    return 1j * (R / (2 * k) - np.exp(1j * k * R) * np.sin(R * k) / (2 * k * k))


def g_free(r, k: float):
    """Free-space outgoing Green function exp(j k r) / (4 pi r), eq. (def:Green)."""
    r = np.asarray(r, dtype=np.float64)
    return np.exp(1j * k * r) / (4.0 * np.pi * r)
