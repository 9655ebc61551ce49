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


def test_far_field_of_a_radial_source_is_the_outgoing_wave():
    # outside a radially symmetric source v(rho) (support rho < a) the convolution with
    # g = exp(ikr)/(4 pi r) is the outgoing spherical wave (exp(ikr)/(kr)) int_0^a v rho sin(k rho) drho
    # (the mean of g over a sphere of radius rho about the origin is g(r) sin(k rho)/(k rho) for
    # r > rho).  The detector operator is the rectangle rule of that convolution on the voxel grid,
    # so h^2 G~ v at the detector pixels must approach it as the grid is refined (a smooth bump:
    # fast convergence).  Physical units: cube side L = 8, detector plane x3 = L, i.e. x_Gamma = n
    # voxels; the voxel-unit operator carries k h, and h^3 sum g(h .) = h^2 sum g~(.).
    from scipy import integrate
    from oracle import bump
    L, kb, a, q = 8.0, 1.3, 2.8, 4
    moment = integrate.quad(lambda r: bump.bump(r, a, q) * r * np.sin(kb * r), 0.0, a, epsabs=1e-15, epsrel=1e-13)[0]
    errs = []
    for n in (8, 16, 32):
        h = L / n
        c = (np.arange(n) - n // 2 + 1) * h
        Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
        v = bump.bump(np.sqrt(X ** 2 + Y ** 2 + Z ** 2), a, q).astype(np.complex128)
        y = h * h * farfield.farfield_fft(v, kb * h, float(n))
        r = np.sqrt(c[:, None] ** 2 + c[None, :] ** 2 + L * L)
        ref = np.exp(1j * kb * r) / (kb * r) * moment
        errs.append(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    assert errs[0] > 30 * errs[1] > 900 * errs[2] and errs[2] < 1e-6, errs
