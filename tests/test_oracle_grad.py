"""Pins for oracle.grad: the conjugated-forward-solve gradient equals the explicit adjoint built
from conjugate transposes, central finite differences, and the dot-product test."""
import numpy as np

from oracle import grad, kernel, ops
from paper_1910_13844_amd import workloads

K = workloads.k_of()


def _setup(n=4, Q=2):
    gm = kernel.gm_coset(n, 4, K)
    prob = grad.Problem(np.fft.fftn(gm), n, K, float(n), tol=1e-14)
    f = workloads.blob_potential(7, n, nblobs=3, sigma_range=(1.0, 2.0), dn_max=0.1)
    dirs = workloads.cone_dirs(Q, 40.0)
    ftrue = f + workloads.blob_potential(8, n, nblobs=2, sigma_range=(1.0, 1.5), dn_max=0.03)
    _, yhat = prob.forward(ftrue, dirs)
    return gm, prob, f, dirs, yhat


def test_adjoint_equals_explicit():
    gm, prob, f, dirs, yhat = _setup()
    loss, g = prob.loss_grad(f, dirs, yhat)
    us, ys = prob.forward(f, dirs)
    rs = ys - yhat
    w = [1.0 / np.vdot(y, y).real for y in yhat]
    ge = grad.grad_explicit(ops.G_dense(gm, 4), f, us, rs, w, K, 4.0)
    assert np.max(np.abs(g - ge)) <= 1e-9 * np.max(np.abs(ge))


def test_gradient_matches_central_differences():
    gm, prob, f, dirs, yhat = _setup()
    loss, g = prob.loss_grad(f, dirs, yhat)
    eps = 1e-5
    rng = np.random.default_rng(0)
    for idx in rng.choice(f.size, 6, replace=False):
        e = np.zeros(f.size)
        e[idx] = eps
        e = e.reshape(f.shape)
        fd = (prob.loss(f + e, dirs, yhat) - prob.loss(f - e, dirs, yhat)) / (2 * eps)
        assert abs(fd - g.ravel()[idx]) <= 1e-6 * np.max(np.abs(g)), (idx, fd, g.ravel()[idx])


def test_dot_product_test():
    # <J df, r>_R = <df, Re J^* r>  with J df from a linearised forward difference of H
    gm, prob, f, dirs, yhat = _setup(Q=1)
    us, ys = prob.forward(f, dirs)
    rng = np.random.default_rng(1)
    df = rng.standard_normal(f.shape)
    r = workloads.random_field(3, ys[0].shape)
    g = prob.vjp(f, us, [r])
    h = 1e-6
    _, yp = prob.forward(f + h * df, dirs)
    _, ym = prob.forward(f - h * df, dirs)
    Jdf = (yp[0] - ym[0]) / (2 * h)
    lhs = np.real(np.vdot(r, Jdf))
    rhs = np.sum(df * g)
    assert abs(lhs - rhs) <= 1e-7 * abs(lhs)
