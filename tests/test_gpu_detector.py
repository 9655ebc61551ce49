"""GPU parity of the detector-side operators (wide far field and its transpose, pupil, decimation)
and of the gradient through the chain against the oracle (oracle.detector), through the C ABI.

Bars: complex128 1e-12 (FP64 pipelines); complex64 2e-6 (single-precision inputs, FP64 inside).
The chained gradient (complex128, solves at 1e-13) 1e-9.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import detector as det  # noqa: E402
from oracle import farfield, kernel  # noqa: E402
from oracle import grad as ograd  # noqa: E402
from paper_1910_13844_amd import api, autograd, workloads  # noqa: E402

K = workloads.k_of()
DEV = "cuda:0"
_ctx = {}


def ctx(n, prec):
    if (n, prec) not in _ctx:
        _ctx[(n, prec)] = api.Context(n, K, p=4, xg=float(n), prec=prec, device=DEV)
    return _ctx[(n, prec)]


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def rnd(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("n,m,prec,tol", [(8, 8, "c128", 1e-12), (8, 16, "c128", 1e-12), (16, 24, "c128", 1e-12),
                                          (32, 64, "c64", 2e-6)])
def test_wide_far_field_and_transpose(n, m, prec, tol):
    c = ctx(n, prec)
    f = workloads.blob_potential(1, n, dn_max=0.05)
    u = rnd((2, n, n, n), 0)
    ft, ut = torch.from_numpy(f).to(DEV, c.rdtype), torch.from_numpy(u).to(DEV, c.cdtype)
    y = c.ls_farfield_wide(m, ft, ut).cpu().numpy()
    fr, ur = ft.cpu().numpy().astype(np.float64), ut.cpu().numpy().astype(np.complex128)
    for q in range(2):
        ref = det.farfield_wide_fft(fr * ur[q], K, float(n), m)
        assert rel(y[q], ref) < tol
    if m == n:   # equals the square-detector path
        ys = c.ls_farfield(ft, ut).cpu().numpy()
        assert rel(y[0], ys[0]) < (1e-12 if prec == "c128" else 2e-6)
    r = rnd((2, m, m), 1)
    rt = torch.from_numpy(r).to(DEV, c.cdtype)
    rr = rt.cpu().numpy().astype(np.complex128)
    for cj in (False, True):
        out = c.ls_farfield_wide_adj(m, rt, conj=cj).cpu().numpy()
        for q in range(2):
            ref = det.farfield_wide_T(np.conj(rr[q]) if cj else rr[q], K, float(n), n)
            assert rel(out[q], ref) < tol


@pytest.mark.parametrize("prec,tol", [("c128", 1e-12), ("c64", 2e-6)])
def test_pupil_and_decimation(prec, tol):
    n, m = 16, 48
    c = ctx(n, prec)
    y = rnd((3, m, m), 2)
    yt = torch.from_numpy(y).to(DEV, c.cdtype)
    yr = yt.cpu().numpy().astype(np.complex128)
    for adj in (False, True):
        out = c.ls_pupil(yt, 0.8, 3.5, adjoint=adj).cpu().numpy()
        ref = det.pupil(yr, K, 0.8, 3.5, adjoint=adj)
        assert rel(out, ref) < tol
    for q in (2, 3):
        d = c.ls_decimate(yt, q).cpu().numpy()
        assert np.array_equal(d, det.decimate(yt.cpu().numpy(), q))
        back = c.ls_decimate(torch.from_numpy(d).to(DEV), q, m=m, transpose=True).cpu().numpy()
        assert np.array_equal(back, det.decimate_T(d, q, m).astype(back.dtype))


def test_chain_gradient_matches_oracle():
    n, m, q, na, dz = 8, 16, 2, 0.7, 2.0
    dirs = workloads.cone_dirs(3, 40.0)
    f0, ft = workloads.perturbed_potential(n)
    prob = ograd.Problem(kernel.ghat_m(n, 4, K), n, K, float(n), tol=1e-13)
    _, yhat = det.chain_forward(prob, ft, dirs, m, na, dz, q)
    us, y = det.chain_forward(prob, f0, dirs, m, na, dz, q)
    g_ref = det.chain_vjp(prob, f0, us, list(y - yhat), m, na, dz, q)
    c = ctx(n, "c128")
    f = torch.from_numpy(f0).to(DEV).requires_grad_(True)
    yg = autograd.detector_fields(f, c, dirs, m, na=na, dz=dz, q=q, tol=1e-13)
    assert rel(yg.detach().cpu().numpy(), y) < 1e-10
    loss = 0.5 * (yg - torch.from_numpy(yhat).to(DEV)).abs().pow(2).sum()
    loss.backward()
    e = rel(f.grad.cpu().numpy(), g_ref)
    print(f"[detector chain] gradient vs oracle {e:.2e}", flush=True)
    assert e < 1e-9
