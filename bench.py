#!/usr/bin/env python
"""Benchmark of the hot path: LS solves/s on the 128^3 x 60-illumination workload.

One step = ls_forward (BiCGSTAB to tol 1e-5 for all 60 plane waves on a 45-degree cone, blob
phantom seed 0, complex64 fields with FP64 reductions) + ls_farfield (128 x 128 detector per
illumination).  Inputs are resident in HBM before the timed region; the one-time Green-kernel
build is timed separately.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK = 78.6   # TFLOP/s: 256 CU x 64 FMA lanes/clk x 2 x 2.4 GHz, non-packed FP32
FP32_PACKED_PEAK = 157.3  # TFLOP/s with packed (2-wide) FP32 FMA; the kernels are compiled without packed FP32


def pct(a, q):
    import numpy as np
    return float(np.percentile(np.asarray(a), q))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="B")
    ap.add_argument("--prof-reps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one device-to-device copy of 1 GiB (reference for rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs on a single MI355X; sharding the illuminations "
              "over several GPUs is not implemented", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1910_13844_amd import _lib, api, workloads

    W = workloads.WORKLOADS[args.workload]
    n, Q = W.n, W.Q
    dev = "cuda:0"
    f_np = W.potential()
    dirs = W.dirs()
    rd = torch.float32 if W.precision == "c64" else torch.float64
    cd = torch.complex64 if W.precision == "c64" else torch.complex128
    f = torch.from_numpy(f_np).to(dev, rd)

    t = time.perf_counter()
    ctx = api.Context(n, W.k, p=W.p, xg=W.xg, prec=W.precision, device=dev)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t
    print(f"[bench] green init n={n}: {t_init * 1e3:.1f} ms", file=sys.stderr, flush=True)

    wsF = ctx.workspace(Q, _lib.LS_OP_FORWARD)
    wsFF = ctx.workspace(Q, _lib.LS_OP_FARFIELD)
    u = torch.empty((Q, n, n, n), dtype=cd, device=dev)
    stream = torch.cuda.current_stream()
    grad_mode = W.kind == "gradient"

    if grad_mode:
        # measured data: fields of the perturbed potential with 30 dB noise (untimed)
        _, f_true = workloads.perturbed_potential(n, W.seed)
        ft = torch.from_numpy(f_true).to(dev, rd)
        ctx.ls_forward(ft, dirs, tol=W.tol, u=u, ws=wsF)
        yhat = torch.from_numpy(workloads.add_noise(ctx.ls_farfield(ft, u, ws=wsFF).cpu().numpy())).to(dev, cd)
        del ft
        wsG = ctx.workspace(Q, _lib.LS_OP_GRAD)

        def step():
            loss, g, info = ctx.ls_grad(f, dirs, yhat, tol=W.tol, ws=wsG)
            return info, g
    else:
        def step():
            _, info = ctx.ls_forward(f, dirs, tol=W.tol, u=u, ws=wsF)
            y = ctx.ls_farfield(f, u, ws=wsFF)
            return info, y

    for i in range(args.warmup):
        step()
        print(f"[bench] warmup {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    times, infos = [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        info, y = step()
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
        infos.append(info)
        print(f"[bench] step {k}: {times[-1]:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    value = (1 if grad_mode else Q) * args.steps / total
    last = infos[-1]
    iters = [i["iters"] for i in last]
    mvs = [i["matvecs"] for i in last]
    relres = [i["relres_true"] for i in last]
    assert all(i["status"] == 0 for i in last), "not all illuminations converged"

    # ---- per-kernel live timing of the four solver passes (HIP events on the launch stream)
    c = 16 if W.precision == "c128" else 8
    N = n ** 3
    Nc = N * c
    ker_bytes = (n + 1) * 4 * n * n * c
    passes = {
        "k_xfwd": (0, Q * 6.5 * Nc, 2),
        "k_yz": (1, Q * 6 * Nc + ker_bytes, 2),
        "k_xinv": (2, Q * 7 * Nc, 2),
        "k_update": (3, Q * 7 * Nc, 1),
    }
    # algorithmic bytes per launch (units of N*c per slot):
    #   k_xfwd (p-update prologue): read r p v (3) + f (0.5), write p (1) + x-spectrum (2)
    #   k_yz   read the x-spectrum (2), write the class-split (y,z) output (4), + kernel once
    #   k_xinv (v epilogue): read the class output (4) + p, rh (2), write v (1)
    #   k_update: read x p s t rh (5), write x r (2)
    # FFT flops of the (y,z) pass with C ky classes of M = 2n/C points (5 L log2 L per L-point
    # transform): per (slot, kx) C x [n forward + n inverse M-point row DFTs + M columns x 4
    # n-point DFTs (z-convolution)] + pointwise kernel products
    import math
    C = {True: {8: 2, 16: 2, 32: 2, 64: 2, 96: 6, 128: 8, 144: 18, 192: 12, 256: 16},
         False: {8: 2, 16: 2, 32: 2, 64: 2, 96: 2, 128: 4, 144: 6, 192: 6, 256: 8}}[W.precision == "c128"][n]
    Mc = 2 * n // C
    yz_flops = Q * 2 * n * C * (2 * n * 5 * Mc * math.log2(Mc) + Mc * 4 * 5 * n * math.log2(n)
                                + 2 * Mc * n * 6)
    prof_ws = torch.empty_like(wsF)
    prof_u = u.clone()
    kern = {}
    for name, (pid, nbytes, per_it) in passes.items():
        api.profile_pass(ctx, f, prof_u, pid, 1, prof_ws)  # warm
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        api.profile_pass(ctx, f, prof_u, pid, args.prof_reps, prof_ws)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.prof_reps
        kern[name] = {"avg_ms": ms, "alg_bytes": nbytes, "gbs": nbytes / (ms * 1e-3) / 1e9,
                      "share": per_it * ms}
    del prof_ws, prof_u
    if args.calib_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    dom = max(kern, key=lambda k: kern[k]["share"])
    dk = kern[dom]
    hbm = {"achieved": round(dk["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(dk["gbs"] / HBM_PEAK_GBS, 4)}
    if dom == "k_yz":
        # the (y,z) pass is limited by vector-ALU issue (transforms in registers and LDS), not HBM
        tf = yz_flops / (dk["avg_ms"] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": round(tf, 2), "peak": FP32_VALU_PEAK, "unit": "TFLOP/s",
                "frac": round(tf / FP32_VALU_PEAK, 4), "traffic": measured_traffic(W.name, dom),
                "alg_flops_per_launch": yz_flops, "alg_bytes_per_launch": dk["alg_bytes"],
                "avg_launch_ms": round(dk["avg_ms"], 4), "frac_of_packed_fp32_peak": round(tf / FP32_PACKED_PEAK, 4),
                "hbm": hbm}
    else:
        roof = {"kernel": dom, "bound": "hbm", **hbm, "traffic": measured_traffic(W.name, dom),
                "alg_bytes_per_launch": dk["alg_bytes"], "avg_launch_ms": round(dk["avg_ms"], 4)}
    per_kernel = {k: {"avg_ms": round(v["avg_ms"], 4), "GB/s": round(v["gbs"], 1),
                      "hbm_frac": round(v["gbs"] / HBM_PEAK_GBS, 4), "traffic": measured_traffic(W.name, k)}
                  for k, v in kern.items()}

    if args.workload == "B":
        metric = "LS solves/sec at 128^3x60 illum, FP32 vs plain at 1e-4 rel err; p50/p99 ms"
    elif grad_mode:
        metric = f"data-term gradients/sec at {n}^3x{Q} views ({W.precision}, tol {W.tol:g}); p50/p99 ms"
    else:
        metric = f"LS solves/sec at {n}^3x{Q} illum ({W.precision}, tol {W.tol:g}); p50/p99 ms"
    solve_ms = [i["time_ms"] for step_info in infos for i in step_info]
    assert min(solve_ms) > 0, "every solve reports its device completion time"
    out = {
        "metric": metric,
        "value": round(value, 3),
        "unit": "gradients/s" if grad_mode else "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * total / args.steps, 2),
        # per-solve completion time over all timed steps: device clock from the batch's first pass
        # to the step at which that illumination's solve reached its final state
        "p50_ms": round(pct(solve_ms, 50), 2),
        "p99_ms": round(pct(solve_ms, 99), 2),
        "step_p50_ms": round(pct(times, 50), 2),
        "step_p99_ms": round(pct(times, 99), 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 fields, f64 reductions" if W.precision == "c64" else "c128",
        "data": data_description(W),
        "config": {"workload": W.name, "n": n, "padded_fft": 2 * n, "illuminations": Q, "group_size": Q, "tol": W.tol,
                   "detector": f"{n}x{n}", "p": W.p, "green_init_ms": round(t_init * 1e3, 1)},
        "solve": {"solves_per_step": len(last), "iters_mean": float(np.mean(iters)), "iters_max": int(max(iters)),
                  "matvecs_mean": float(np.mean(mvs)), "relres_true_max": float(max(relres))},
        "roofline": roof,
        "kernels": per_kernel,
    }

    if not args.no_cpu_baseline:
        if grad_mode:   # fields of f0 for the oracle's residual check (u held the data fields)
            ctx.ls_forward(f, dirs, tol=W.tol, u=u, ws=wsF)
        out["cpu_baseline"], out["oracle_check"] = cpu_baseline(W, f_np, dirs, u, float(np.mean(mvs)),
                                                                per_step=len(last), grad_mode=grad_mode)
    print(json.dumps(out), flush=True)
    return 0


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or
    None when that summary is missing or was taken from a different kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    src = os.path.join(ROOT, "paper_1910_13844_amd", "csrc")
    try:
        sha = hashlib.sha256(open(os.path.join(src, "kernels.hip"), "rb").read() +
                            open(os.path.join(src, "fft.hpp"), "rb").read()).hexdigest()[:16]
        vals = {}
        for line in open(path):
            if ":" in line and not line.startswith("|"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
        if vals.get("kernel_source_sha256_16") != sha:
            return None
        return float(vals[f"traffic_bytes_per_launch {kernel}"])
    except (OSError, KeyError, ValueError):
        return None


def data_description(W):
    if W.phantom == "sphere":
        return "synthetic (homogeneous sphere, radius 10 voxels, index 1.36; one plane wave along +z)"
    return (f"synthetic (seeded 20-blob phantom, dn <= {W.dn_max}; {W.Q} plane waves on a "
            f"{W.theta_deg:g}-degree cone)")


def host_description():
    """The host the oracle is timed on: logical CPUs visible to this process and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_baseline(W, f_np, dirs, u, mv_per_solve, per_step=1, grad_mode=False):
    """The FP64 oracle timed on the host: one application of A = I - G diag f at the full size
    (two FFTs of (2n)^3) and one far field, scaled by the matvecs per solve of the GPU run.  The
    same matvec gives the oracle's residual of the GPU solution for illumination 0."""
    import numpy as np

    from oracle import farfield as ofar
    from oracle import incident, kernel, ops

    n = W.n
    t = time.perf_counter()
    gh = kernel.ghat_m(n, W.p, W.k)
    t_setup = time.perf_counter() - t
    u0 = u[0].cpu().numpy().astype(np.complex128)
    b = incident.plane_wave(n, W.k, dirs[0])
    t = time.perf_counter()
    Au = ops.A_apply(gh, f_np, u0)
    t_mv = time.perf_counter() - t
    relres = float(np.linalg.norm(b - Au) / np.linalg.norm(b))
    t = time.perf_counter()
    ofar.farfield_fft(f_np * u0, W.k, W.xg)
    t_ff = time.perf_counter() - t
    per_solve = t_mv * mv_per_solve + t_ff
    if grad_mode:   # one gradient = per_step solves (forward and adjoint of every view)
        base = {"value": round(1.0 / (per_solve * per_step), 8), "unit": "gradients/s", "cores": 1, "kind": "oracle",
                "host": host_description(), "sample": (f"1 FP64 application of A (2 FFTs of {2 * n}^3, numpy) = {t_mv:.2f} s and 1 far field = "
                           f"{t_ff:.2f} s, scaled by {mv_per_solve:.1f} matvecs/solve x {per_step} solves/gradient; "
                           f"kernel setup {t_setup:.1f} s excluded")}
        return base, {"oracle_relres_q0": relres, "tol": W.tol}
    base = {"value": round(1.0 / per_solve, 6), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "host": host_description(), "sample": (f"1 FP64 application of A (2 FFTs of {2 * n}^3, numpy) = {t_mv:.2f} s and 1 far field = "
                       f"{t_ff:.2f} s, scaled by {mv_per_solve:.1f} matvecs/solve; kernel setup {t_setup:.1f} s "
                       "excluded")}
    check = {"oracle_relres_q0": relres, "tol": W.tol}
    return base, check


if __name__ == "__main__":
    sys.exit(main())
