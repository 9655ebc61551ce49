"""Pins for oracle.ops: the four forms of G agree exactly; G is complex symmetric; G converges
to the continuous convolution g * v as in Theorem 1."""
import numpy as np
import pytest

from oracle import kernel, ops, bump
from paper_1910_13844_amd import workloads

K = 1.0469375


def rand(n, seed=0):
    return workloads.random_field(seed, (n, n, n))


@pytest.mark.parametrize("n,p", [(6, 4), (8, 4), (8, 2)])
def test_prop2_equals_theorem1(n, p):
    v = rand(n)
    a = ops.G_fft(kernel.ghat_m(n, p, K), v)
    b = ops.G_theorem1(n, p, K, v)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_fft_equals_direct_sum():
    n, p = 6, 4
    v = rand(n, 1)
    gm = kernel.gm_coset(n, p, K)
    a = ops.G_fft(np.fft.fftn(gm), v)
    b = ops.G_direct(gm, v)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_dense_matrix_and_symmetry():
    n, p = 4, 4
    gm = kernel.gm_coset(n, p, K)
    Gd = ops.G_dense(gm, n)
    v = rand(n, 2)
    a = (Gd @ v.ravel()).reshape(v.shape)
    b = ops.G_fft(np.fft.fftn(gm), v)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
    assert np.max(np.abs(Gd - Gd.T)) <= 1e-15 * np.max(np.abs(Gd))


def test_bilinear_symmetry_fft_form():
    n, p = 8, 4
    gh = kernel.ghat_m(n, p, K)
    x, y = rand(n, 3), rand(n, 4)
    lhs = np.sum(x * ops.G_fft(gh, y))
    rhs = np.sum(y * ops.G_fft(gh, x))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_point_sample_matches_fft():
    n, p = 8, 4
    gm = kernel.gm_coset(n, p, K)
    v = rand(n, 5)
    full = ops.G_fft(np.fft.fftn(gm), v)
    for pt in [(0, 0, 0), (7, 3, 5), (4, 4, 4)]:
        assert abs(ops.G_point(gm, v, *pt) - full[pt]) <= 1e-12 * np.max(np.abs(full))


def _bump_errors(n, p, L=8.0, kb=1.3, a=2.8, q=4):
    h = L / n
    c = (np.arange(n) - n // 2 + 1) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    v = bump.bump(np.sqrt(X ** 2 + Y ** 2 + Z ** 2), a, q).astype(np.complex128)
    Gv = h * h * ops.G_fft(kernel.ghat_m(n, p, kb * h), v)
    e = 0.0
    for (x, y, z) in [(0.0, 0.0, 0.0), (1.0, 1.0, -1.0), (2.0, -1.0, 1.0)]:
        i = tuple(int(round(t / h)) + n // 2 - 1 for t in (z, y, x))
        ref = bump.conv_exact(np.sqrt(x * x + y * y + z * z), kb, a, q)
        e = max(e, abs(Gv[i] - ref) / abs(ref))
    return e


def test_convergence_to_continuous_convolution():
    # Theorem 1 error bound: physical cube of side L = 8, radial bump of radius a = 0.35 L with
    # q = 4.  With h = L/n the voxel-unit kernel uses k h and G_phys = h^2 G_voxel.  The error at
    # grid points falls quickly with n at p = 4, and p = 2 leaves the trapezoid error C/p^2
    # (the remark that p should be at least 4).
    errs = [_bump_errors(n, 4) for n in (8, 16, 32)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-6
    assert _bump_errors(32, 2) > 100 * errs[2]
