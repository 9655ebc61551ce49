"""Full-size parity on the 128^3 workloads (through the C ABI).

128^3 x 60 illuminations (blob phantom seed 0, 45-degree cone, tol 1e-5, complex64): the oracle
cannot solve 60 systems of 2M unknowns in a test, so the FP64 GPU path is pinned to it instead --
solved to 1e-10, its residual measured with the oracle's own operator at q in {0, 15, 30, 45} --
and every complex64 solution and detector field is compared with that FP64 solution (bar 1e-4).

Gradient workload (f0 = phantom seed 2, f_true = f0 + 5-blob perturbation seed 3, 40 views on a
40-degree cone, 30 dB noise seed 4): oracle gradient at n = 32 with the same construction, and
central differences (step 1e-3 in f) at 50 voxels drawn by default_rng(5) at n = 128.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import farfield, incident, kernel, ops  # noqa: E402
from oracle import grad as ograd  # noqa: E402
from paper_1910_13844_amd import api, workloads  # noqa: E402

K = workloads.k_of()
DEV = "cuda:0"


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_config_B_fp32_within_1e4_of_oracle_pinned_fp64():
    W = workloads.WORKLOADS["B"]
    n = W.n
    f = W.potential()
    dirs = W.dirs()
    c64 = api.Context(n, K, p=W.p, xg=W.xg, prec="c64", device=DEV)
    f32 = torch.from_numpy(f.astype(np.float32)).to(DEV)
    u32, i32 = c64.ls_forward(f32, dirs, tol=W.tol)
    y32 = c64.ls_farfield(f32, u32).cpu().numpy()
    u32 = u32.cpu().numpy()
    del c64
    torch.cuda.empty_cache()
    c128 = api.Context(n, K, p=W.p, xg=W.xg, prec="c128", device=DEV)
    f64 = torch.from_numpy(f).to(DEV)
    u64, i64 = c128.ls_forward(f64, dirs, tol=1e-10)
    y64 = c128.ls_farfield(f64, u64).cpu().numpy()
    u64 = u64.cpu().numpy()
    del c128
    torch.cuda.empty_cache()
    assert all(i["status"] == 0 for i in i32 + i64)
    print(f"[B] iters c64 mean {np.mean([i['iters'] for i in i32]):.1f}, "
          f"c128 mean {np.mean([i['iters'] for i in i64]):.1f}", flush=True)

    # pin the FP64 reference: the oracle's operator and far field applied to it
    print("[oracle] ghat_m n=128 p=4", flush=True)
    gh = kernel.ghat_m(n, W.p, K)
    kern = farfield.slice_kernels(n, K, W.xg)
    for q in (0, 15, 30, 45):
        b = incident.plane_wave(n, K, dirs[q])
        rr = np.linalg.norm(b - ops.A_apply(gh, f, u64[q])) / np.linalg.norm(b)
        ey = rel(y64[q], farfield.farfield_fft(f * u64[q], K, W.xg, kern))
        print(f"[oracle] q={q} residual {rr:.2e}, far field {ey:.2e}", flush=True)
        assert rr < 2e-10 and ey < 1e-12, (q, rr, ey)

    eu = [rel(u32[q], u64[q]) for q in range(W.Q)]
    ey = [rel(y32[q], y64[q]) for q in range(W.Q)]
    print(f"[B] complex64 vs FP64: u max {max(eu):.2e}, y max {max(ey):.2e}", flush=True)
    assert max(eu) < 1e-4 and max(ey) < 1e-4


def _d_problem(n):
    f0, ft = workloads.perturbed_potential(n)
    dirs = workloads.cone_dirs(40, 40.0)
    return f0, ft, dirs


def test_config_D_gradient_vs_oracle_n32():
    n = 32
    f0, ft, dirs = _d_problem(n)
    prob = ograd.Problem(kernel.ghat_m(n, 4, K), n, K, float(n), tol=1e-11)
    print("[oracle] forward for the data", flush=True)
    _, y = prob.forward(ft, dirs)
    yhat = workloads.add_noise(y)
    print("[oracle] loss and gradient", flush=True)
    lo, go = prob.loss_grad(f0, dirs, yhat)
    # what the solver tolerance alone costs: the FP64 oracle stopped at the workload's tolerance
    # (1e-6) instead of 1e-11
    W = workloads.WORKLOADS["D"]
    _, go6 = ograd.Problem(prob.ghat_m, n, K, float(n), tol=W.tol).loss_grad(f0, dirs, yhat)
    print(f"[D n=32] oracle gradient at tol {W.tol:g} vs 1e-11: {rel(go6, go):.2e}", flush=True)
    # complex64 at the workload's tolerance must meet the FP32 target: 1e-4 from the tight oracle
    for prec, tol, bar_l, bar_g in (("c128", 1e-11, 1e-9, 1e-8), ("c64", W.tol, 1e-4, 1e-4)):
        c = api.Context(n, K, p=4, xg=float(n), prec=prec, device=DEV)
        rd = torch.float64 if prec == "c128" else torch.float32
        cd = torch.complex128 if prec == "c128" else torch.complex64
        loss, g, info = c.ls_grad(torch.from_numpy(f0).to(DEV, rd), dirs, torch.from_numpy(yhat).to(DEV, cd), tol=tol)
        e = rel(g.cpu().numpy(), go)
        print(f"[D n=32 {prec}] loss {loss:.8e} vs {lo:.8e}, gradient rel {e:.2e}", flush=True)
        assert all(i["status"] == 0 for i in info)
        assert abs(loss - lo) <= bar_l * lo and e < bar_g


def test_config_D_central_differences_n128():
    n = 128
    f0, ft, dirs = _d_problem(n)
    c = api.Context(n, K, p=4, xg=float(n), prec="c128", device=DEV)
    tol = 1e-12

    def fields(fv):
        ftt = torch.from_numpy(fv).to(DEV)
        u, info = c.ls_forward(ftt, dirs, tol=tol)
        assert all(i["status"] == 0 for i in info)
        return c.ls_farfield(ftt, u)

    # data from the same operator (this test checks the gradient against the loss it differentiates)
    yhat = torch.from_numpy(workloads.add_noise(fields(ft).cpu().numpy())).to(DEV)
    loss0, g, info = c.ls_grad(torch.from_numpy(f0).to(DEV), dirs, yhat, tol=tol)
    g = g.cpu().numpy().ravel()
    nyh = (yhat.abs() ** 2).sum(dim=(1, 2))

    def loss(fv):
        r = fields(fv) - yhat
        return float(((r.abs() ** 2).sum(dim=(1, 2)) / (2 * nyh)).sum())

    idx = np.random.default_rng(5).choice(n ** 3, 50, replace=False)
    eps = 1e-3
    fd = np.empty(50)
    for j, i in enumerate(idx):
        fp, fm = f0.copy().ravel(), f0.copy().ravel()
        fp[i] += eps
        fm[i] -= eps
        fd[j] = (loss(fp.reshape(f0.shape)) - loss(fm.reshape(f0.shape))) / (2 * eps)
    e = np.linalg.norm(fd - g[idx]) / np.linalg.norm(g[idx])
    print(f"[D n=128 FD] loss {loss0:.6e}, |g| range {np.abs(g[idx]).min():.2e}..{np.abs(g[idx]).max():.2e}, "
          f"FD rel {e:.2e}, max abs {np.abs(fd - g[idx]).max():.2e}", flush=True)
    assert e < 1e-4
