"""Pins of the detector-side operators (oracle.detector).

Wide far field: equals the brute-force double sum for m > n; equals the already pinned square
detector (oracle.farfield) when m = n; its central n x n pixels equal the square detector's for any
m (same positions, same sum); its transpose satisfies the bilinear identity.  Pupil: identity when
the pupil covers the whole grid and dz = 0; adjoint identity; never increases energy; its impulse
response at dz = 0 is the Airy pattern of a disk of radius na k (pins the cutoff); it carries the
field of a beamed source from x_Gamma to x_Gamma + dz as the far-field sum at the farther plane gives
it (pins the sign and wavenumber of the propagation phase).  Decimation:
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


def test_pupil_impulse_response_is_the_airy_pattern():
    # at dz = 0 the pupil is the ideal low-pass of radius W = na k: the response to one pixel is the
    # inverse transform of a disk, W J1(W r) / (2 pi r) (W^2 / (4 pi) at r = 0) up to the sampling of
    # the disk on the 2m frequency grid, which shrinks as m grows.  A cutoff at na k0 (the vacuum
    # wavenumber) would scale the central value by 1 / 1.333^2.
    from scipy import special
    k = workloads.k_of()
    for na in (0.5, 1.0):
        W = na * k
        errs = []
        for m in (64, 128):
            y = np.zeros((m, m), dtype=np.complex128)
            a0 = m // 2 - 1
            y[a0, a0] = 1.0
            out = det.pupil(y, k, na, 0.0)
            pos = np.arange(m) - a0
            R = np.sqrt(pos[:, None] ** 2 + pos[None, :] ** 2)
            airy = W * W / (4 * np.pi) * np.ones_like(R)
            nz = R > 0
            airy[nz] = W * special.j1(W * R[nz]) / (2 * np.pi * R[nz])
            sel = R <= 12
            errs.append(np.max(np.abs(out[sel] - airy[sel])) / airy.max())
        assert errs[1] < errs[0] < 1e-2 and errs[1] < 3e-3, (na, errs)


def test_pupil_propagates_the_field_to_the_next_plane():
    # a field that solves the homogeneous Helmholtz equation beyond the detector plane is carried
    # from x3 = x_Gamma to x3 = x_Gamma + dz by multiplying its angular spectrum with
    # exp(+i dz sqrt(k^2 - |w|^2)).  The far field of a source beamed along the axis (a Gaussian
    # envelope times exp(i k x3), little energy near the cutoff |w| = k) computed at x_Gamma and sent
    # through the pupil (na = 1) must therefore match the far field computed directly at
    # x_Gamma + dz, on the central half of a wide detector (finite window).  The opposite sign, or
    # the vacuum wavenumber in the cutoff, gives errors of order 1 or 1e-1.
    k = workloads.k_of()
    n, m, sig, xg, dz = 16, 64, 3.0, 10.0, 4.0
    c = np.arange(n) - n // 2 + 1.0
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    for th in (0.0, 0.3):
        v = np.exp(-(X ** 2 + Y ** 2 + Z ** 2) / (2 * sig ** 2)) * np.exp(1j * k * (np.sin(th) * X + np.cos(th) * Z))
        y1 = det.farfield_wide_fft(v, k, xg, m)
        y2 = det.farfield_wide_fft(v, k, xg + dz, m)
        yp = det.pupil(y1, k, 1.0, dz)
        cc = slice(m // 4, 3 * m // 4)
        e = np.linalg.norm((yp - y2)[cc, cc]) / np.linalg.norm(y2[cc, cc])
        assert e < 2e-3, (th, e)
