"""GPU tests of the torch.autograd.Function and of the continuous-batching loop.

autograd: backward through ls_vjp equals the oracle gradient (c128, 1e-9) and passes
torch.autograd.gradcheck on a small grid.  Serving: every request served in a mixed stream gets
exactly the result of the same request computed alone (forward: ls_forward + ls_farfield;
gradient: ls_grad) -- slots never interact.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from oracle import grad as ograd  # noqa: E402
from oracle import kernel  # noqa: E402
from paper_1910_13844_amd import api, autograd, serve, workloads  # noqa: E402

K = workloads.k_of()
DEV = "cuda:0"


def test_autograd_backward_matches_oracle_gradient():
    n = 8
    c = api.Context(n, K, p=4, xg=float(n), prec="c128", device=DEV)
    f0 = workloads.blob_potential(2, n, nblobs=4, sigma_range=(1.5, 3.0), dn_max=0.05)
    pert = workloads.blob_potential(3, n, nblobs=2, sigma_range=(1.0, 2.0), dn_max=0.01)
    dirs = workloads.cone_dirs(3, 40.0)
    prob = ograd.Problem(kernel.ghat_m(n, 4, K), n, K, float(n), tol=1e-13)
    _, yhat = prob.forward(f0 + pert, dirs)
    f = torch.from_numpy(f0).to(DEV).requires_grad_(True)
    y = autograd.farfield(f, c, dirs, tol=1e-13)
    loss = autograd.data_loss(y, torch.from_numpy(yhat).to(DEV), c)
    loss.backward()
    lo, go = prob.loss_grad(f0, dirs, yhat)
    assert abs(loss.item() - lo) <= 1e-10 * lo
    g = f.grad.cpu().numpy()
    assert np.linalg.norm(g - go) / np.linalg.norm(go) < 1e-9


def test_autograd_gradcheck():
    n = 8
    c = api.Context(n, K, p=4, xg=float(n), prec="c128", device=DEV)
    f0 = workloads.blob_potential(5, n, nblobs=3, sigma_range=(1.5, 3.0), dn_max=0.05)
    dirs = workloads.cone_dirs(2, 40.0)
    f = torch.from_numpy(f0).to(DEV).requires_grad_(True)
    fn = lambda x: autograd.farfield(x, c, dirs, tol=1e-14, maxit=2000)  # noqa: E731
    assert torch.autograd.gradcheck(fn, (f,), eps=1e-6, atol=1e-8, rtol=1e-5, fast_mode=True)


@pytest.mark.parametrize("scheduler", ["single", "concurrent"])
def test_served_results_equal_alone(scheduler):
    # single: pools stepped one after the other; concurrent: one host thread and stream per pool
    trace = serve.poisson_trace(6, 1000.0, [16, 32], qmax=4, seed=3)
    eng = serve.GpuEngine(hbm_budget_gb=4.0, tol=1e-6, max_slots=5)
    eng.preload(trace)
    sch = (serve.Scheduler if scheduler == "single" else serve.ConcurrentScheduler)(eng, iters_per_step=1)
    res = sch.run(trace, realtime=False)
    assert res["requests"] == len(trace)
    for r in trace:
        c = eng.ctx[r.n]
        d = eng.data.get(r.rid) or {}
        f = torch.from_numpy(workloads.blob_potential(r.seed, r.n, dn_max=0.05)).to(DEV, c.rdtype)
        dirs = workloads.cone_dirs(r.Q, r.theta)
        if r.kind == "forward":
            u, _ = c.ls_forward(f, dirs, tol=1e-6)
            y = c.ls_farfield(f, u)
            assert torch.equal(y, r.outputs["y"]), r.rid
        else:
            pert = workloads.blob_potential(r.seed + 100000, r.n, nblobs=5, sigma_range=(2.0, 5.0), dn_max=0.01)
            ft = torch.from_numpy(workloads.blob_potential(r.seed, r.n, dn_max=0.05) + pert).to(DEV, c.rdtype)
            ut, _ = c.ls_forward(ft, dirs, tol=1e-6)
            ym = c.ls_farfield(ft, ut)
            loss, g, _ = c.ls_grad(f, dirs, ym, tol=1e-6)
            assert abs(loss - r.outputs["loss"]) <= 1e-12 * abs(loss)
            assert torch.equal(g, r.outputs["grad"]), r.rid
