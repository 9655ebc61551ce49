"""Pins of the incident-field propagation (oracle.incident.angular_spectrum), Section "Computation of
the 3D Incident Field" and Fig. 3.

A plane wave is an exact solution of free-space propagation, so a detector field that samples one
must come back as that plane wave in the whole volume: exactly when its lateral frequency is on the
DFT grid (with or without tilt transfer), and still exactly with tilt transfer when it is not
(the amplitude a is then constant), while plain periodic propagation then errs (the Fig. 3
experiment).  Also: zero distance is the identity on band-limited fields, propagation composes
(z1 then z2 equals z1 + z2), and evanescent components are dropped.
"""
import numpy as np
import pytest

from oracle import incident
from paper_1910_13844_amd import workloads

K = workloads.k_of()


def plane_wave_at_detector(n, k, kt, xg):
    """y_in and the exact volume of the plane wave exp(i(k~.x~ + kz x3))."""
    kx, ky = kt
    kz = np.sqrt(k * k - kx * kx - ky * ky)
    c = np.arange(n, dtype=np.float64) - n // 2 + 1
    lat = np.exp(1j * (kx * c[None, :] + ky * c[:, None]))
    y_in = lat * np.exp(1j * kz * xg)
    vol = lat[None, :, :] * np.exp(1j * kz * c)[:, None, None]
    return y_in, vol


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("tilt", [True, False])
def test_on_grid_plane_wave_is_exact(tilt):
    n = 16
    kt = (2 * np.pi * 2 / n, -2 * np.pi * 1 / n)   # DFT frequencies
    y_in, vol = plane_wave_at_detector(n, K, kt, float(n))
    u = incident.angular_spectrum(y_in, K, float(n), kt, tilt_transfer=tilt)
    assert rel(u, vol) < 1e-13


def test_tilt_transfer_fig3():
    # off-grid tilt, 30 degrees from the axis: exact with tilt transfer, visibly wrong without
    n = 32
    th, ph = np.deg2rad(30.0), np.deg2rad(20.0)
    kt = (K * np.sin(th) * np.cos(ph), K * np.sin(th) * np.sin(ph))
    y_in, vol = plane_wave_at_detector(n, K, kt, float(n))
    with_tt = incident.angular_spectrum(y_in, K, float(n), kt, tilt_transfer=True)
    without = incident.angular_spectrum(y_in, K, float(n), kt, tilt_transfer=False)
    assert np.max(np.abs(with_tt - vol)) < 1e-12
    assert np.max(np.abs(without - vol)) > 0.05


def test_zero_distance_identity_and_composition():
    n = 16
    rng = np.random.default_rng(0)
    spec = np.fft.fft2(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    spec *= np.abs(incident.propagator(n, K, 0.0)) > 0          # band-limit to |w| <= k
    y = np.fft.ifft2(spec)
    p0 = incident.propagator(n, K, 0.0)
    assert np.allclose(np.fft.ifft2(np.fft.fft2(y) * p0), y, atol=1e-14)
    p1, p2, p12 = (incident.propagator(n, K, d) for d in (2.5, 4.0, 6.5))
    assert np.allclose(p1 * p2, p12, atol=1e-14)


def test_evanescent_dropped():
    n = 16
    p = incident.propagator(n, K, 3.0)
    w = incident.lateral_freqs(n)
    r2 = w[:, None] ** 2 + w[None, :] ** 2
    assert np.all(p[r2 > K * K] == 0) and np.allclose(np.abs(p[r2 <= K * K]), 1.0)
