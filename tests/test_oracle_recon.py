"""Pins of the reconstruction oracle: TV prox (oracle.tv) and accelerated FBS (oracle.recon).

TV prox: adjointness of the difference operators, TV of known fields, the closed forms of the
prox for lam = 0, constant inputs and two voxels, and the duality gap (a certificate that does not
depend on how the dual point was found).  FBS: on nonnegative least squares (whose minimiser
scipy.optimize.nnls gives) the loop with gamma_k = gamma_0 / sqrt(k) converges to that minimiser.
"""
import numpy as np
import pytest
import scipy.optimize as so

from oracle import kernel, recon, tv
from oracle import grad as ograd
from paper_1910_13844_amd import workloads


def test_diff_adjoint():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((5, 6, 7))
    p = rng.standard_normal((3, 5, 6, 7))
    assert abs(np.vdot(tv.diff(x), p) - np.vdot(x, tv.diff_T(p))) < 1e-12


def test_tv_known_fields():
    n = 6
    assert tv.tv(np.full((n, n, n), 2.5)) == 0.0
    step = np.zeros((n, n, n))
    step[: n // 2] = 1.0                          # one jump of height 1 across an n x n face
    assert abs(tv.tv(step) - n * n) < 1e-12
    ramp = np.broadcast_to(np.arange(n, dtype=float)[None, None, :], (n, n, n)).copy()
    assert abs(tv.tv(ramp) - n * n * (n - 1)) < 1e-12   # unit slope along x, last column has no difference
    # isotropic: a diagonal ramp x + y has |grad| = sqrt(2) where both differences exist
    diag = np.add.outer(np.zeros(n), np.add.outer(np.arange(n), np.arange(n))).astype(float)
    expect = n * ((n - 1) ** 2 * np.sqrt(2.0) + 2 * (n - 1))
    assert abs(tv.tv(diag) - expect) < 1e-9


def test_prox_special_cases():
    rng = np.random.default_rng(1)
    b = rng.standard_normal((4, 5, 6))
    assert np.array_equal(tv.fgp_prox(b, 0.0, 10, True), np.maximum(b, 0.0))
    assert np.array_equal(tv.fgp_prox(b, 0.0, 10, False), b)
    c = np.full((4, 4, 4), 0.7)
    assert np.allclose(tv.fgp_prox(c, 0.5, 50, True), c, atol=1e-14)
    assert np.array_equal(tv.fgp_prox(-np.abs(b) - 0.1, 0.3, 100, True), np.zeros_like(b))


@pytest.mark.parametrize("b0,b1,lam", [(1.0, 0.2, 0.1), (1.0, 0.2, 0.5), (0.3, 2.0, 0.25), (-0.5, 0.5, 0.2)])
def test_prox_two_voxels_closed_form(b0, b1, lam):
    # TV of two voxels is |x0 - x1|: soft-threshold the difference by 2 lam, keep the mean
    b = np.array([b0, b1]).reshape(2, 1, 1)
    mean, half = (b0 + b1) / 2, (b0 - b1) / 2
    h = np.sign(half) * max(abs(half) - lam, 0.0)
    expect = np.array([mean + h, mean - h])
    x = tv.fgp_prox(b, lam, 2000, nonneg=False).ravel()
    assert np.allclose(x, expect, atol=1e-9)
    if expect.min() >= 0:
        assert np.allclose(tv.fgp_prox(b, lam, 2000, nonneg=True).ravel(), expect, atol=1e-9)


@pytest.mark.parametrize("nonneg", [True, False])
def test_prox_duality_gap_closes(nonneg):
    rng = np.random.default_rng(2)
    b = 0.5 * rng.standard_normal((6, 6, 6)) + 0.3
    lam = 0.3
    gaps = []
    for it in (50, 500, 3000):
        x, p = tv.fgp_prox(b, lam, it, nonneg, return_dual=True)
        gaps.append(tv.dual_gap(b, lam, p, nonneg))
    assert all(g >= -1e-9 for g in gaps)
    assert gaps[1] < gaps[0] / 10 and gaps[2] < gaps[1] / 3
    assert gaps[2] < 1e-6 * tv.primal(x, b, lam)


def test_fbs_converges_to_nnls():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((30, 12))
    y = rng.standard_normal(30)
    xs, _ = so.nnls(A, y)
    L = np.linalg.norm(A, 2) ** 2
    f = recon.fbs(np.zeros(12), lambda v, s: A.T @ (A @ v - y), lambda z, g: np.maximum(z, 0.0), 1.0 / L,
                  [[0]] * 4000)
    assert np.linalg.norm(f - xs) / np.linalg.norm(xs) < 1e-6


def test_reconstruct_decreases_objective():
    # tiny Lippmann-Schwinger problem: the objective falls from the starting point
    n, Q = 8, 6
    K = workloads.k_of()
    f0, ft = workloads.perturbed_potential(n)
    dirs = workloads.cone_dirs(Q, 40.0)
    prob = ograd.Problem(kernel.ghat_m(n, 4, K), n, K, float(n), tol=1e-12)
    _, y = prob.forward(ft, dirs)
    tau = 1e-4

    def objective(f):
        return prob.loss(f, dirs, list(y)) + tau * tv.tv(f)

    subs = workloads.view_subsets(Q, 3, 10, seed=7)
    start = np.zeros((n, n, n))
    f = recon.reconstruct(prob, dirs, list(y), start, tau, 30.0, subs, tv_iters=50)
    assert f.min() >= 0.0
    # 10 stochastic iterations from f = 0: objective 3.0 -> ~6e-3, error to the true potential ~0.15
    assert objective(f) < 0.01 * objective(start)
    assert np.linalg.norm(f - ft) / np.linalg.norm(ft) < 0.3
