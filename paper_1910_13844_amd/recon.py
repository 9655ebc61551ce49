"""Reconstruction loop: accelerated forward-backward splitting (Algorithm 1, Section "Optimization").

Each iteration k evaluates the data-term gradient over a subset of the views at the extrapolated
point v^k (ls_grad: forward solves, far fields, residuals, adjoint solves, accumulation), takes the
proximal step f^k = prox_{gamma_k tau TV + i_{>=0}}(v^k - gamma_k d^k) with gamma_k = gamma_0 / sqrt(k)
(ls_prox_tv, fast gradient projection on the dual), and extrapolates
v^{k+1} = f^k + ((a_k - 1) / a_{k+1}) (f^k - f^{k-1}) (ls_fbs_extrapolate).  The host only keeps
the scalars a_k, gamma_k and the subsets; every array operation runs in libls.

With warm starts the gradient is assembled from the same building blocks ls_grad runs internally
(forward solves, far field, residual, transposed far field, adjoint solves, accumulation), and
every forward BiCGSTAB run starts from the total field u_q that view's previous solve returned
(kept per view on the device) instead of from the incident field; optionally the adjoint solves
start from their previous solution w_q as well.  The stopping test is the same (relative residual against the right-hand
side), so the iterates agree with the cold-started loop to the solver tolerance; between
neighbouring iterates f changes little, so the solves need fewer iterations.

    python -m paper_1910_13844_amd.recon [--n 128] [--views 40] [--iters 10] [--subset 8] [--warm-start]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from .api import Context


class WarmGradient:
    """Data-term gradient over a subset of views with warm-started solves.  Holds, per view, the
    total field u_q and the adjoint field w_q of its last solve ([Q, n, n, n] each, device); both
    are first computed at f0 with cold starts (one gradient over all views)."""

    def __init__(self, ctx: Context, dirs, y_meas: torch.Tensor, f0: torch.Tensor, tol: float,
                 adjoint: bool = True):
        self.ctx, self.tol, self.adjoint = ctx, tol, adjoint
        self.dirs = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
        self.y_meas = y_meas
        self.u, _ = ctx.ls_forward(f0, self.dirs, tol=tol)
        self.w = None
        if adjoint:
            r, _, _ = ctx.ls_residual(ctx.ls_farfield(f0, self.u), y_meas)
            self.w, _ = ctx.ls_forward_uin(f0, ctx.ls_farfield_adj(r, conj=True), tol=tol)

    def __call__(self, v: torch.Tensor, sub: Sequence[int]):
        """(loss, gradient, solve info) at v over the views `sub`, as ls_grad returns them."""
        c = self.ctx
        idx = torch.as_tensor(list(sub), dtype=torch.long, device=self.u.device)
        u, i_fw = c.ls_forward(v, self.dirs[list(sub)], tol=self.tol, u=self.u.index_select(0, idx),
                               warm_start=True)
        y = c.ls_farfield(v, u)
        r, stats, loss = c.ls_residual(y, self.y_meas.index_select(0, idx), out=y)
        b = c.ls_farfield_adj(r, conj=True)
        if self.adjoint:
            w, i_ad = c.ls_forward_uin(v, b, tol=self.tol, u=self.w.index_select(0, idx), warm_start=True)
            self.w.index_copy_(0, idx, w)
        else:
            w, i_ad = c.ls_forward_uin(v, b, tol=self.tol)
        grad = c.ls_grad_accumulate(u, w, torch.empty_like(v), stats=stats)
        self.u.index_copy_(0, idx, u)
        return float(loss), grad, i_fw + i_ad


def reconstruct(ctx: Context, dirs, y_meas: torch.Tensor, f0: torch.Tensor, tau: float, gamma0: float,
                subsets: Sequence[Sequence[int]], tv_iters: int, tol: float = 1e-5, nonneg: bool = True,
                history: Optional[List[dict]] = None, f_ref: Optional[torch.Tensor] = None,
                warm_start: bool = False, warm_adjoint: bool = False) -> torch.Tensor:
    """Algorithm 1 for len(subsets) iterations.  dirs [Q, 3] (host), y_meas [Q, n, n] (device),
    f0 [n]^3 (device, the context's real type).  Returns f^K.  With `history`, one record per
    iteration; with `f_ref` as well, each record holds ||f^k - f_ref|| / ||f_ref||.  warm_start:
    gradients by WarmGradient (its set-up at f0 runs before the first iteration); warm_adjoint:
    whether the adjoint solves start from their previous solution too (else from the right-hand
    side: the adjoint right-hand side follows the data residual, which changes direction and size
    between visits of a view, and measured at 128^3 the previous solution saves no iterations)."""
    dirs = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
    f_prev = f0.clone()
    v = f0.clone()
    f = torch.empty_like(f0)
    a = 1.0
    ws_prox = ctx.workspace(1, _lib.LS_OP_PROX)
    warm = WarmGradient(ctx, dirs, y_meas, f0, tol, warm_adjoint) if warm_start else None
    for k, sub in enumerate(subsets, start=1):
        sub = list(sub)
        gamma = gamma0 / math.sqrt(k)
        t0 = time.perf_counter()
        if warm is not None:
            loss, d, info = warm(v, sub)
        else:
            loss, d, info = ctx.ls_grad(v, dirs[sub], y_meas[sub].contiguous(), tol=tol)
        ctx.ls_prox_tv(v, gamma * tau, tv_iters, d=d, gamma=gamma, nonneg=nonneg, out=f, ws=ws_prox)
        a_next = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * a * a))
        ctx.ls_fbs_extrapolate(f, f_prev, (a - 1.0) / a_next, out=v)
        f_prev, f = f, f_prev
        a = a_next
        if history is not None:
            torch.cuda.synchronize()
            rec = {"k": k, "loss_at_v": loss, "gamma": gamma, "views": sub, "seconds": time.perf_counter() - t0,
                   "iters": [i["iters"] for i in info]}
            if f_ref is not None:
                rec["rel_err"] = float((f_prev - f_ref).norm() / f_ref.norm())
            history.append(rec)
    return f_prev


def lipschitz_estimate(ctx: Context, dirs, y_meas: torch.Tensor, f0: torch.Tensor, iters: int = 8,
                       seed: int = 0) -> float:
    """Largest eigenvalue of sum_q Re(J_q^* J_q) / ||y_q||^2 at f0 = 0 by power iteration (the
    Lipschitz constant of the data-term gradient of the linearised model).  Algorithm 1 leaves
    gamma_0 free; 1 / L scaled to the subset size is the default step of ``main``.  J_q df is the far
    field of df . u_in,q (ls_farfield) and J_q^* r one adjoint solve (ls_vjp), both at f0 = 0
    where the solves are the identity."""
    dirs = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
    zero = torch.zeros_like(f0)
    u, _ = ctx.ls_forward(zero, dirs, tol=1e-6)
    w = (y_meas.abs() ** 2).sum(dim=(1, 2)).to(ctx.cdtype).reshape(-1, 1, 1)
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.rand(f0.shape, generator=g, dtype=torch.float64).to(f0.device, f0.dtype)
    lam = 0.0
    for _ in range(iters):
        x = x / x.norm()
        jx = ctx.ls_farfield(x, u)
        hx, _ = ctx.ls_vjp(zero, u, (jx / w).contiguous(), tol=1e-6)
        lam = float((hx * x).sum())
        x = hx
    return lam


def main(argv=None) -> int:
    """Reconstruct the gradient workload's perturbed phantom from its simulated measurements."""
    from . import workloads

    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--views", type=int, default=40)
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--subset", type=int, default=8)
    ap.add_argument("--tau", type=float, default=1e-4)
    ap.add_argument("--gamma0", type=float, default=None,
                    help="initial step; default 1 / L of the subset's linearised data term")
    ap.add_argument("--tv-iters", type=int, default=50)
    ap.add_argument("--prec", default="c64")
    ap.add_argument("--warm-start", action="store_true",
                    help="start every solve from that view's previous solution (set-up at f0 included in the time)")
    args = ap.parse_args(argv)
    dev = "cuda:0"
    n, Q = args.n, args.views
    ctx = Context(n, workloads.k_of(), p=4, xg=float(n), prec=args.prec, device=dev)
    _, f_true = workloads.perturbed_potential(n)
    dirs = workloads.cone_dirs(Q, 40.0)
    ft = torch.from_numpy(f_true).to(dev, ctx.rdtype)
    u, _ = ctx.ls_forward(ft, dirs, tol=1e-6)
    y = torch.from_numpy(workloads.add_noise(ctx.ls_farfield(ft, u).cpu().numpy())).to(dev, ctx.cdtype)
    del u
    subs = workloads.view_subsets(Q, args.subset, args.iters, seed=7)
    f_start = torch.zeros_like(ft)
    L_full = lipschitz_estimate(ctx, dirs, y, f_start)
    gamma0 = args.gamma0 if args.gamma0 is not None else Q / (args.subset * L_full)
    hist: List[dict] = []
    torch.cuda.synchronize()
    t = time.perf_counter()
    f = reconstruct(ctx, dirs, y, f_start, args.tau, gamma0, subs, args.tv_iters, history=hist,
                    warm_start=args.warm_start)
    torch.cuda.synchronize()
    total = time.perf_counter() - t
    # a second, untimed run that records the error to the truth after every iteration
    hist_err: List[dict] = []
    reconstruct(ctx, dirs, y, f_start, args.tau, gamma0, subs, args.tv_iters, history=hist_err, f_ref=ft,
                warm_start=args.warm_start)
    marks = sorted({k for k in (1, 2, 5, 10, 20, 50, 100, 200, 500, 1000, 2000) if k <= args.iters} | {args.iters})
    err = float((f - ft).norm() / ft.norm())
    print(json.dumps({"n": n, "views": Q, "iters": args.iters, "subset": args.subset, "warm_start": args.warm_start,
                      "lipschitz": L_full,
                      "gamma0": gamma0, "tau": args.tau, "tv_iters": args.tv_iters, "seconds": total,
                      "seconds_per_iter": total / args.iters, "rel_err_to_truth": err,
                      "rel_err_at": {k: hist_err[k - 1]["rel_err"] for k in marks},
                      "loss_at_v_at": {k: hist[k - 1]["loss_at_v"] for k in marks},
                      "solver_iters_mean_at": {k: float(np.mean(hist[k - 1]["iters"])) for k in marks}}),
          flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
