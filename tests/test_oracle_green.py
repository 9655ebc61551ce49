"""Pins for oracle.green: the Fourier transform of the truncated Green function.

eqs. (GreenL) and (GreenL2) of the paper, checked against direct 1D quadrature of the radial
integral (1/s) int_0^R exp(j k r) sin(s r) dr, which is the definition of the transform of a
radial function truncated at R.
"""
import numpy as np
import pytest
from scipy import integrate

from oracle import green


def quad_ghat(s, k, R):
    if s == 0.0:
        fr = lambda r: r * np.cos(k * r)
        fi = lambda r: r * np.sin(k * r)
        sc = 1.0
    else:
        fr = lambda r: np.cos(k * r) * np.sin(s * r)
        fi = lambda r: np.sin(k * r) * np.sin(s * r)
        sc = 1.0 / s
    lim = 2000
    re = integrate.quad(fr, 0, R, limit=lim, epsabs=1e-12, epsrel=1e-12)[0]
    im = integrate.quad(fi, 0, R, limit=lim, epsabs=1e-12, epsrel=1e-12)[0]
    return sc * complex(re, im)


@pytest.mark.parametrize("k,n", [(1.0469375, 8), (1.0469375, 16), (2.3, 12)])
def test_ghat_matches_quadrature(k, n):
    R = np.sqrt(3.0) * n
    rng = np.random.default_rng(0)
    ss = np.concatenate([[0.0, 0.5 * k, k * (1 - 1e-9), 2 * k, np.pi], rng.uniform(0.01, np.pi, 6)])
    got = green.ghat_t(ss, k, R)
    for s, g in zip(ss, got):
        ref = quad_ghat(float(s), k, R)
        assert abs(g - ref) <= 1e-9 * max(1.0, abs(ref)), (s, g, ref)


def test_value_on_sphere_equals_greenL2():
    for k, n in [(1.0469375, 8), (0.7, 32), (2.9, 64)]:
        R = np.sqrt(3.0) * n
        a = green.ghat_t(np.array([k]), k, R)[0]
        b = green.ghat_t_at_k(k, R)
        assert abs(a - b) <= 1e-12 * abs(b)


def test_zero_frequency_limit():
    k, R = 1.0469375, np.sqrt(3.0) * 16
    g0 = green.ghat_t(np.array([0.0]), k, R)[0]
    g_eps = green.ghat_t(np.array([1e-6]), k, R)[0]
    assert abs(g0 - g_eps) <= 1e-6 * abs(g0)
    assert abs(g0 - quad_ghat(0.0, k, R)) <= 1e-10 * abs(g0)


def test_corrected_greenL_agrees_and_printed_sign_does_not():
    k, n = 1.0469375, 8
    R = np.sqrt(3.0) * n
    s = np.array([0.1, 0.4, 0.8, 1.5, 2.5, 3.0])
    ref = green.ghat_t(s, k, R)
    corr = green.ghat_t_printed(s, k, R, sign=-1)
    printed = green.ghat_t_printed(s, k, R, sign=+1)
    assert np.max(np.abs(corr - ref) / np.abs(ref)) < 1e-12
    # the printed sign gives values off by O(1): the sign reading is forced
    assert np.max(np.abs(printed - ref) / np.abs(ref)) > 1e-2


def test_large_argument_decay_bound():
    # |ghat_t(w)| <= 2 / ((|w| - k) |w|) for |w| > k (bound used in the proof of Theorem 1)
    k, R = 1.0469375, np.sqrt(3.0) * 64
    s = np.linspace(1.2, 40.0, 200)
    g = np.abs(green.ghat_t(s, k, R))
    assert np.all(g <= 2.0 / ((s - k) * s) + 1e-15)
