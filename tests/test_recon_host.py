"""Host logic of the warm-started gradient (recon.WarmGradient) with a stand-in context on the CPU:
each view's cached field is the one handed to its next solve as the initial guess, the solve's
result replaces exactly that view's entry, and the loss is the data term of eq. (prob) from the
residual statistics."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1910_13844_amd import recon  # noqa: E402

n = 4


class FakeCtx:
    """Solves return the initial guess plus the view's direction tag (u) or the right-hand side
    plus one (w); the far field sums the volume along z; everything else is bookkeeping."""

    def __init__(self):
        self.guesses = []

    def ls_forward(self, f, dirs, tol, u=None, warm_start=False):
        dirs = np.asarray(dirs).reshape(-1, 3)
        tag = torch.from_numpy(dirs[:, 0].copy()).to(torch.complex128).reshape(-1, 1, 1, 1)
        base = u.clone() if warm_start else torch.zeros((len(dirs), n, n, n), dtype=torch.complex128)
        if warm_start:
            self.guesses.append(("u", u.clone()))
        return base + tag, [{"iters": 1}] * len(dirs)

    def ls_farfield(self, f, u):
        return u.sum(dim=1)

    def ls_residual(self, y, y_meas, out=None):
        r = y - y_meas
        stats = torch.stack([torch.stack([(ri.abs() ** 2).sum(), (mi.abs() ** 2).sum()]) for ri, mi in zip(r, y_meas)])
        if out is not None:
            out.copy_(r)
            r = out
        st = stats.reshape(-1).to(torch.float64)
        return r, st, (st[0::2] / (2 * st[1::2])).sum()

    def ls_farfield_adj(self, r, conj=False):
        return (r.conj() if conj else r).unsqueeze(1).expand(-1, n, -1, -1).contiguous()

    def ls_forward_uin(self, f, b, tol, u=None, warm_start=False):
        if warm_start:
            self.guesses.append(("w", u.clone()))
            return u + 1.0, [{"iters": 2}] * b.shape[0]
        return b + 1.0, [{"iters": 3}] * b.shape[0]

    def ls_grad_accumulate(self, u, w, grad, stats=None):
        wq = 1.0 / stats[1::2] if stats is not None else torch.ones(u.shape[0], dtype=torch.float64)
        grad.copy_(sum(wq[q] * (u[q] * w[q]).real for q in range(u.shape[0])))
        return grad


@pytest.mark.parametrize("adjoint", [False, True])
def test_warm_gradient_caches_per_view(adjoint):
    Q = 5
    dirs = np.zeros((Q, 3))
    dirs[:, 0] = np.arange(1, Q + 1)          # view q's solve adds q + 1
    rng = np.random.default_rng(0)
    y_meas = torch.from_numpy(rng.standard_normal((Q, n, n)) + 1j * rng.standard_normal((Q, n, n)))
    f = torch.zeros((n, n, n), dtype=torch.float64)
    ctx = FakeCtx()
    wg = recon.WarmGradient(ctx, dirs, y_meas, f, 1e-5, adjoint=adjoint)
    u0 = wg.u.clone()
    assert torch.equal(u0[:, 0, 0, 0].real, torch.arange(1, Q + 1, dtype=torch.float64))
    sub = [3, 0]
    loss, grad, info = wg(f, sub)
    kind, guess = ctx.guesses[0]
    assert kind == "u" and torch.equal(guess, u0[sub])            # the cached fields of views 3 and 0
    for q in range(Q):                                              # only those views move on
        moved = q in sub
        assert torch.equal(wg.u[q], u0[q] + (q + 1) if moved else u0[q])
    u = u0[sub] + torch.tensor([4.0, 1.0], dtype=torch.complex128).reshape(-1, 1, 1, 1)
    r = u.sum(dim=1) - y_meas[sub]
    want = sum(float((r[i].abs() ** 2).sum() / (2 * (y_meas[q].abs() ** 2).sum())) for i, q in enumerate(sub))
    assert loss == pytest.approx(want, rel=1e-14)
    assert len(info) == 2 * len(sub)
    if adjoint:
        assert ctx.guesses[1][0] == "w" and torch.equal(ctx.guesses[1][1] + 1.0, wg.w[sub])
    else:
        assert wg.w is None and len(ctx.guesses) == 1
