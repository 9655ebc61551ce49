"""Pins for oracle.kernel: Proposition 2's coset-sum kernel equals the restriction of the
Theorem 1 inverse DFT on the np grid to the 2n grid (an exact algebraic identity), and the
kernel has the symmetries of a radial function sampled on a cube."""
import numpy as np
import pytest

from oracle import kernel, green

K = 1.0469375


@pytest.mark.parametrize("n,p", [(8, 2), (8, 4), (8, 6), (6, 8), (16, 4)])
def test_coset_sum_equals_np_grid_crop(n, p):
    a = kernel.gm_coset(n, p, K)
    b = kernel.gm_direct(n, p, K)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))


def test_p2_is_plain_inverse_dft():
    n = 8
    gm = kernel.gm_coset(n, 2, K)
    M = 2 * n
    q = kernel.signed(M).astype(float)
    s = (2 * np.pi / M) * np.sqrt(q[:, None, None] ** 2 + q[None, :, None] ** 2 + q[None, None, :] ** 2)
    ref = np.fft.ifftn(green.ghat_t(s, K, np.sqrt(3.0) * n))
    assert np.max(np.abs(gm - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_kernel_even_and_cubic_symmetric():
    n, p = 8, 4
    gm = kernel.gm_coset(n, p, K)
    neg = (-np.arange(2 * n)) % (2 * n)
    assert np.max(np.abs(gm - gm[np.ix_(neg, neg, neg)])) < 1e-15
    assert np.max(np.abs(gm - np.transpose(gm, (1, 0, 2)))) < 1e-15
    assert np.max(np.abs(gm - np.transpose(gm, (2, 1, 0)))) < 1e-15
    gh = np.fft.fftn(gm)
    assert np.max(np.abs(gh - gh[np.ix_(neg, neg, neg)])) < 1e-12 * np.max(np.abs(gh))


def test_kernel_approximates_green_function_away_from_origin():
    # gm[k] ~ g(|k|) for |k| >> 1 inside the truncation radius (Theorem 1 quadrature limit);
    # the agreement improves with p (trapezoid error term C/p^2).
    n = 16
    errs = []
    for p in (2, 4):
        gm = kernel.gm_direct(n, p, K)
        pts = [(5, 0, 0), (0, 7, 3), (4, 4, 4), (9, 2, 1)]
        e = 0
        for pt in pts:
            r = np.sqrt(sum(t * t for t in pt))
            ref = green.g_free(r, K)
            e = max(e, abs(gm[pt] - ref) / abs(ref))
        errs.append(e)
    assert errs[1] < 0.2
    assert errs[1] < errs[0]
