"""Pins for oracle.farfield: the padded-FFT form equals the brute-force double sum, the transpose
is the exact transpose, and the far field of a weak radial source matches the continuous
outgoing-wave formula as the grid is refined."""
import numpy as np

from oracle import farfield, green
from paper_1910_13844_amd import workloads

K = workloads.k_of()


def test_fft_form_equals_brute_force():
    n = 6
    v = workloads.random_field(0, (n, n, n))
    a = farfield.farfield_fft(v, K, float(n))
    b = farfield.farfield_direct(v, K, float(n))
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_transpose_is_exact():
    n = 6
    v = workloads.random_field(1, (n, n, n))
    r = workloads.random_field(2, (n, n))
    lhs = np.sum(r * farfield.farfield_fft(v, K, float(n)))
    rhs = np.sum(v * farfield.farfield_T(r, K, float(n)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    a = farfield.farfield_T(r, K, float(n))
    b = farfield.farfield_T_direct(r, K, float(n))
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_single_voxel_source_is_green_function():
    # v = delta at voxel (iz, iy, ix): y[a] = g(a - b, x_Gamma - k3) exactly
    n = 8
    v = np.zeros((n, n, n), dtype=complex)
    v[2, 5, 1] = 1.0
    y = farfield.farfield_fft(v, K, float(n))
    c = np.arange(n) - n // 2 + 1
    Z = n - c[2]
    dy = c[:, None] - c[5]
    dx = c[None, :] - c[1]
    ref = green.g_free(np.sqrt(dy ** 2 + dx ** 2 + Z ** 2), K)
    assert np.max(np.abs(y - ref)) <= 1e-14 * np.max(np.abs(ref))
