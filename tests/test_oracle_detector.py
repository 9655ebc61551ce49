"""Pins of the detector-side operators (oracle.detector).

Wide far field: equals the brute-force double sum for m > n; equals the already pinned square
detector (oracle.farfield) when m = n; its central n x n pixels equal the square detector's for any
m (same positions, same sum); its transpose satisfies the bilinear identity.  Pupil: identity when
the pupil covers the whole grid and dz = 0; adjoint identity; never increases energy.  Decimation:
keeps the pixel at the lateral origin; adjoint identity.
"""
import numpy as np
import pytest

from oracle import detector as det
from oracle import farfield
from paper_1910_13844_amd import workloads

K = workloads.k_of()


def rnd(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("n,m", [(4, 4), (4, 8), (6, 10), (4, 6)])
def test_wide_far_field_equals_direct_sum(n, m):
    v = rnd((n, n, n), 0)
    xg = float(n)
    a = det.farfield_wide_fft(v, K, xg, m)
    b = det.farfield_wide_direct(v, K, xg, m)
    assert np.allclose(a, b, rtol=0, atol=1e-12 * np.abs(b).max())


def test_square_detector_and_central_pixels():
    n = 8
    v = rnd((n, n, n), 1)
    xg = float(n)
    sq = farfield.farfield_fft(v, K, xg)
    assert np.allclose(det.farfield_wide_fft(v, K, xg, n), sq, atol=1e-12 * np.abs(sq).max())
    for m in (12, 16):
        w = det.farfield_wide_fft(v, K, xg, m)
        s = (m - n) // 2
        assert np.allclose(w[s:s + n, s:s + n], sq, atol=1e-12 * np.abs(sq).max())


@pytest.mark.parametrize("n,m", [(6, 6), (6, 12)])
def test_wide_transpose_identity(n, m):
    v = rnd((n, n, n), 2)
    r = rnd((m, m), 3)
    lhs = np.sum(det.farfield_wide_fft(v, K, float(n), m) * r)
    rhs = np.sum(v * det.farfield_wide_T(r, K, float(n), n))
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_pupil_identity_adjoint_energy():
    m = 16
    y = rnd((2, m, m), 4)
    assert np.allclose(det.pupil(y, K, 10.0, 0.0), y, atol=1e-13)      # pupil covers every frequency
    x = rnd((m, m), 5)
    z = rnd((m, m), 6)
    px = det.pupil(x, K, 0.8, 3.0)
    assert abs(np.vdot(px, z) - np.vdot(x, det.pupil(z, K, 0.8, 3.0, adjoint=True))) < 1e-12 * np.linalg.norm(x) ** 2
    assert np.linalg.norm(px) <= np.linalg.norm(x) * (1 + 1e-12)
    assert np.linalg.norm(det.pupil(x, K, 0.3, 0.0)) < 0.5 * np.linalg.norm(x)   # white noise loses most energy


def test_decimation():
    m, q = 12, 3
    y = rnd((m, m), 7)
    d = det.decimate(y, q)
    o = m // 2 - 1                                   # index of the pixel at lateral position 0
    assert d.shape == (m // q, m // q)
    assert d[(o - det.decimation_offset(m, q)) // q, (o - det.decimation_offset(m, q)) // q] == y[o, o]
    z = rnd(d.shape, 8)
    assert abs(np.sum(d * z) - np.sum(y * det.decimate_T(z, q, m))) < 1e-12


def test_chain_gradient_central_differences():
    # loss 1/2 sum_q ||B y_q(f) - yhat_q||^2 through the whole chain; gradient vs central differences
    from oracle import grad as ograd
    from oracle import kernel
    n, m, q, na, dz = 6, 10, 2, 0.7, 2.0
    dirs = workloads.cone_dirs(2, 40.0)
    prob = ograd.Problem(kernel.ghat_m(n, 4, K), n, K, float(n), tol=1e-13)
    f0, ft = workloads.perturbed_potential(n)
    _, yhat = det.chain_forward(prob, ft, dirs, m, na, dz, q)

    def loss(f):
        _, y = det.chain_forward(prob, f, dirs, m, na, dz, q)
        return 0.5 * float(np.sum(np.abs(y - yhat) ** 2))

    us, y = det.chain_forward(prob, f0, dirs, m, na, dz, q)
    g = det.chain_vjp(prob, f0, us, list(y - yhat), m, na, dz, q)
    rng = np.random.default_rng(11)
    eps = 1e-5
    for idx in rng.choice(n ** 3, 6, replace=False):
        e = np.zeros(n ** 3)
        e[idx] = eps
        e = e.reshape(f0.shape)
        fd = (loss(f0 + e) - loss(f0 - e)) / (2 * eps)
        assert abs(fd - g.ravel()[idx]) <= 1e-6 * np.abs(g).max(), (idx, fd, g.ravel()[idx])
