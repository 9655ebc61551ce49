#!/usr/bin/env python
"""Benchmark of the hot path: LS solves/s on the 128^3 x 60-illumination workload.

One step = ls_forward_farfield: BiCGSTAB to tol 1e-5 for all 60 plane waves on a 45-degree cone
(blob phantom seed 0, complex64 fields with FP64 reductions) and the far field of every solution
(128 x 128 detector per illumination).  Inputs are resident in HBM before the timed region; the one-time Green-kernel
build is timed separately.  Prints one JSON line whose headline is that workload; the same line
carries the 256^3 x 60 forward workload, the 128^3 x 40-view gradient workload and a 100-request
serving trace (continuous batching against one illumination at a time) as sub-objects
(`configs`), the accuracy of the timed batch against the complex128 path, and the
FP64 oracle timed on the host (`cpu_baseline`).

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--workload B] [--no-extras] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK = 78.6   # TFLOP/s: 256 CU x 64 FMA lanes/clk x 2 x 2.4 GHz, non-packed FP32
FP32_PACKED_PEAK = 157.3  # TFLOP/s with packed (2-wide) FP32 FMA; the kernels are compiled without packed FP32
ACC_QS = (0, 15, 30, 45)  # illuminations compared with the complex128 path


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pct(a, q):
    import numpy as np
    return float(np.percentile(np.asarray(a), q))


def rel(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def classes(n, c128):
    """ky classes of the (y,z) plane pass (ClassCfg in kernels.hip)."""
    return {True: {8: 2, 16: 2, 32: 2, 64: 2, 96: 6, 128: 8, 144: 18, 192: 12, 256: 16},
            False: {8: 2, 16: 2, 32: 2, 64: 4, 96: 4, 128: 4, 144: 6, 192: 6, 256: 8}}[c128][n]


def pass_model(n, Q, c128):
    """Algorithmic bytes (and the plane pass's flops) per launch of the four solver passes.

    Bytes in units of N*c per slot (f, shared by the slots, counted once per launch):
      k_xfwd (p-update prologue): read r p v (3), write p (1) + x-spectrum (2) = 6, + f
      k_yz   read the x-spectrum (2), write the class-split (y,z) output (4) = 6, + kernel once
      k_xinv (v epilogue): read the class output (4) + p, rh (2), write v (1) = 7
      k_update: read x p s t rh (5), write x r (2) = 7
    Plane-pass flops, the per-illumination count of the (y, z) transforms of a padded 3D FFT
    convolution: 12 n^2 pencils of 2n points (y forward and inverse over the 2n kx planes, 2 x 2n^2;
    z forward and inverse over 2n x 2n (kx, ky), 2 x 4n^2) at 5 L log2 L flops per L-point
    transform.  Also returned: the pruned count of what the kernel computes with C ky classes of
    M = 2n/C points (zero padding skipped): per (slot, kx) C x [n forward + n inverse M-point row
    DFTs + M columns x 4 n-point DFTs (z-convolution)] + 6 flops per kernel product."""
    c = 16 if c128 else 8
    Nc = n ** 3 * c
    f_bytes = n ** 3 * c // 2
    ker_bytes = (n + 1) * 4 * n * n * c
    C = classes(n, c128)
    Mc = 2 * n // C
    yz_pruned = Q * 2 * n * C * (2 * n * 5 * Mc * math.log2(Mc) + Mc * 4 * 5 * n * math.log2(n) + 2 * Mc * n * 6)
    yz_flops = Q * 12 * n * n * 5 * (2 * n) * math.log2(2 * n)
    return {"k_xfwd": (0, Q * 6 * Nc + f_bytes, 2), "k_yz": (1, Q * 6 * Nc + ker_bytes, 2),
            "k_xinv": (2, Q * 7 * Nc, 2), "k_update": (3, Q * 7 * Nc, 1)}, (yz_flops, yz_pruned)


def time_passes(ctx, f, u, ws, n, Q, c128, reps):
    """Average launch time of each solver pass, HIP events on the stream the passes run on."""
    import torch

    from paper_1910_13844_amd import api
    model, yz_flops = pass_model(n, Q, c128)
    stream = torch.cuda.current_stream()
    kern = {}
    for name, (pid, nbytes, per_it) in model.items():
        api.profile_pass(ctx, f, u, pid, 1, ws)  # warm
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        api.profile_pass(ctx, f, u, pid, reps, ws)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        kern[name] = {"avg_ms": ms, "alg_bytes": nbytes, "gbs": nbytes / (ms * 1e-3) / 1e9, "share": per_it * ms}
    return kern, yz_flops


def timed_steps(step, steps, warmup, tag):
    import torch
    stream = torch.cuda.current_stream()
    for i in range(warmup):
        step()
        log(f"{tag} warmup {i} done")
    torch.cuda.synchronize()
    times, infos, out = [], [], None
    t0 = time.perf_counter()
    for k in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        info, out = step()
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
        infos.append(info)
        log(f"{tag} step {k}: {times[-1]:.1f} ms")
    torch.cuda.synchronize()
    return time.perf_counter() - t0, times, infos, out


def load_library(dev="cuda:0"):
    """Loads the library's kernels on the device (the first context of a process pays for that)
    with a tiny grid, so that the timed kernel builds below measure the build alone; returns ms."""
    import torch

    from paper_1910_13844_amd import api, workloads
    torch.zeros(1, device=dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    api.Context(8, workloads.k_of(), p=4, xg=8.0, prec="c64", device=dev)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t)


def forward_workload(W, steps, warmup, dev="cuda:0"):
    """ls_forward_farfield over the whole batch of workload W; returns timings, the last step's
    fields and the context (the caller frees them)."""
    import torch

    from paper_1910_13844_amd import _lib, api
    n, Q = W.n, W.Q
    rd = torch.float32 if W.precision == "c64" else torch.float64
    cd = torch.complex64 if W.precision == "c64" else torch.complex128
    f = torch.from_numpy(W.potential()).to(dev, rd)
    t = time.perf_counter()
    ctx = api.Context(n, W.k, p=W.p, xg=W.xg, prec=W.precision, device=dev)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t
    log(f"green init n={n}: {t_init * 1e3:.1f} ms")
    dirs = W.dirs()
    wsF = ctx.workspace(Q, _lib.LS_OP_FORWARD)
    u = torch.empty((Q, n, n, n), dtype=cd, device=dev)
    y = torch.empty((Q, n, n), dtype=cd, device=dev)

    def step():
        _, _, info = ctx.ls_forward_farfield(f, dirs, tol=W.tol, u=u, y=y, ws=wsF)
        return info, y

    total, times, infos, y = timed_steps(step, steps, warmup, W.name)
    last = infos[-1]
    assert all(i["status"] == 0 for i in last), "not all illuminations converged"
    return {"ctx": ctx, "f": f, "u": u, "y": y, "wsF": wsF, "t_init": t_init, "total": total, "times": times,
            "infos": infos, "dirs": dirs}


def solve_summary(infos):
    import numpy as np
    last = infos[-1]
    iters = [i["iters"] for i in last]
    return {"solves_per_step": len(last), "iters_mean": float(np.mean(iters)), "iters_max": int(max(iters)),
            "matvecs_mean": float(np.mean([i["matvecs"] for i in last])),
            "restarts": int(sum(i["restarts"] for i in last)),
            "relres_true_max": float(max(i["relres_true"] for i in last))}


def accuracy_vs_c128(W, r, dev="cuda:0"):
    """Relative L2 error of the timed batch's fields (illuminations ACC_QS) against the complex128
    path solved to 1e-10 (whose agreement with the FP64 oracle is a parity test)."""
    import torch

    from paper_1910_13844_amd import api
    ctx = api.Context(W.n, W.k, p=W.p, xg=W.xg, prec="c128", device=dev)
    f64 = torch.from_numpy(W.potential()).to(dev)
    d = r["dirs"][list(ACC_QS)]
    u64, info = ctx.ls_forward(f64, d, tol=1e-10)
    y64 = ctx.ls_farfield(f64, u64)
    eu = [rel(r["u"][q].cpu().numpy().astype("complex128"), u64[i].cpu().numpy()) for i, q in enumerate(ACC_QS)]
    ey = [rel(r["y"][q].cpu().numpy().astype("complex128"), y64[i].cpu().numpy()) for i, q in enumerate(ACC_QS)]
    del ctx, u64, y64
    return {"reference": "complex128 path, tol 1e-10", "illuminations": list(ACC_QS),
            "u_rel_l2_max": max(eu), "y_rel_l2_max": max(ey), "u_rel_l2": eu, "y_rel_l2": ey,
            "ref_iters": [i["iters"] for i in info]}


def release(d=None):
    """Drops the device buffers held in dict d (if given) and returns cached blocks to the device."""
    import gc

    import torch
    if d is not None:
        d.clear()
    gc.collect()
    torch.cuda.empty_cache()


def config_C(steps, warmup, reps):
    from paper_1910_13844_amd import workloads
    W = workloads.WORKLOADS["C"]
    r = forward_workload(W, steps, warmup)
    kern, _ = time_passes(r["ctx"], r["f"], r["u"].clone(), r["wsF"], W.n, W.Q, False, reps)
    s = solve_summary(r["infos"])
    out = {"workload": W.name, "n": W.n, "padded_fft": 2 * W.n, "illuminations": W.Q, "tol": W.tol,
           "value": round(W.Q * steps / r["total"], 3), "unit": "solves/s",
           "ms_per_step": round(1e3 * r["total"] / steps, 2), "steps": steps, "warmup": warmup,
           "iters_per_solve": s["iters_mean"], "solve": s, "green_init_ms": round(r["t_init"] * 1e3, 1),
           "passes": {k: {"avg_ms": round(v["avg_ms"], 4), "GB/s": round(v["gbs"], 1),
                          "hbm_frac": round(v["gbs"] / HBM_PEAK_GBS, 4)} for k, v in kern.items()}}
    release(r)
    return out


def config_D(steps, warmup, dev="cuda:0"):
    import numpy as np
    import torch

    from paper_1910_13844_amd import _lib, api, workloads
    W = workloads.WORKLOADS["D"]
    n, Q = W.n, W.Q
    ctx = api.Context(n, W.k, p=W.p, xg=W.xg, prec=W.precision, device=dev)
    f0, f_true = workloads.perturbed_potential(n, W.seed)
    f = torch.from_numpy(f0).to(dev, torch.float32)
    ft = torch.from_numpy(f_true).to(dev, torch.float32)
    dirs = W.dirs()
    u, _ = ctx.ls_forward(ft, dirs, tol=W.tol)
    yhat = torch.from_numpy(workloads.add_noise(ctx.ls_farfield(ft, u).cpu().numpy())).to(dev, torch.complex64)
    del u, ft
    wsG = ctx.workspace(Q, _lib.LS_OP_GRAD)

    def step():
        loss, g, info = ctx.ls_grad(f, dirs, yhat, tol=W.tol, ws=wsG)
        return info, (loss, g)

    total, times, infos, (loss, g) = timed_steps(step, steps, warmup, W.name)
    info = infos[-1]
    assert all(i["status"] == 0 for i in info)
    it = [i["iters"] for i in info]
    out = {"workload": W.name, "n": n, "views": Q, "tol": W.tol, "value": round(steps / total, 3),
           "unit": "gradients/s", "ms_per_step": round(1e3 * total / steps, 2), "steps": steps, "warmup": warmup,
           "solves_per_gradient": len(info), "iters_mean": float(np.mean(it)), "loss": loss,
           "accuracy": "gradient vs the FP64 oracle solved to 1e-11 (n = 32, same construction): "
                       "tests/test_gpu_workloads.py bar 1e-4"}
    del ctx, wsG, f, yhat, g
    release()
    return out


def config_E(requests=100):
    """Serving: a seeded Poisson trace of forward and gradient requests over grid sizes 64-192
    (1-60 illuminations each, 20 requests/s), served with continuous batching and admission by
    device-memory footprint, and the same requests one illumination at a time."""
    from paper_1910_13844_amd import serve
    res = serve.benchmark(requests=requests, baseline=True, progress=0)
    cont, alone = res["continuous"], res["one_at_a_time"]
    out = {"workload": f"serve_trace{requests}_c64", "requests": requests,
           "value": round(cont["solves_per_s"], 2), "unit": "solves/s",
           "p50_ms": round(cont["p50_ms"], 1), "p99_ms": round(cont["p99_ms"], 1),
           "one_at_a_time": {"value": round(alone["solves_per_s"], 2), "p50_ms": round(alone["p50_ms"], 1),
                             "p99_ms": round(alone["p99_ms"], 1)},
           "speedup": round(cont["solves_per_s"] / alone["solves_per_s"], 3),
           "results_equal_alone_vs_mix_max_rel": res["alone_vs_mix_max_rel"],
           "memory": cont["memory"], "trace": res["config"]}
    release()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="B", choices=["A", "B", "C", "D"],
                    help="headline workload; D prints only the gradient workload's object (for profiling)")
    ap.add_argument("--prof-reps", type=int, default=5)
    ap.add_argument("--no-extras", action="store_true", help="headline workload only (no configs, no accuracy)")
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

    from paper_1910_13844_amd import workloads

    if args.workload == "D":
        d = config_D(args.steps, args.warmup)
        W = workloads.WORKLOADS["D"]
        out = {"metric": f"data-term gradients/sec at {W.n}^3 x {W.Q} views (c64, tol {W.tol:g})",
               "value": d["value"], "unit": "gradients/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
               "ms_per_step": d["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "c64 fields, f64 reductions",
               "data": "synthetic (seeded blob phantom f0 and perturbation, 40 plane waves on a 40-degree cone, "
                       "30 dB noise)",
               "config": {k: d[k] for k in ("workload", "n", "views", "tol")},
               "gradient": {k: d[k] for k in ("solves_per_gradient", "iters_mean", "loss", "accuracy")}}
        print(json.dumps(out), flush=True)
        return 0
    W = workloads.WORKLOADS[args.workload]
    n, Q = W.n, W.Q
    c128 = W.precision == "c128"
    lib_ms = load_library()
    r = forward_workload(W, args.steps, args.warmup)
    value = Q * args.steps / r["total"]
    s = solve_summary(r["infos"])

    # ---- per-kernel live timing of the four solver passes (HIP events on the launch stream)
    kern, yz_flops = time_passes(r["ctx"], r["f"], r["u"].clone(), torch.empty_like(r["wsF"]), n, Q, c128,
                                 args.prof_reps)
    if args.calib_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
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
        flops, pruned = yz_flops
        tf = flops / (dk["avg_ms"] * 1e-3) / 1e12
        tfp = pruned / (dk["avg_ms"] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": round(tf, 2), "peak": FP32_VALU_PEAK, "unit": "TFLOP/s",
                "frac": round(tf / FP32_VALU_PEAK, 4), "traffic": measured_traffic(W.name, dom),
                "alg_flops_per_launch": flops, "alg_bytes_per_launch": dk["alg_bytes"],
                "avg_launch_ms": round(dk["avg_ms"], 4), "frac_of_packed_fp32_peak": round(tf / FP32_PACKED_PEAK, 4),
                "pruned_flops_per_launch": pruned, "achieved_pruned": round(tfp, 2),
                "frac_pruned": round(tfp / FP32_VALU_PEAK, 4), "hbm": hbm}
    else:
        roof = {"kernel": dom, "bound": "hbm", **hbm, "traffic": measured_traffic(W.name, dom),
                "alg_bytes_per_launch": dk["alg_bytes"], "avg_launch_ms": round(dk["avg_ms"], 4)}
    per_kernel = {k: {"avg_ms": round(v["avg_ms"], 4), "GB/s": round(v["gbs"], 1),
                      "hbm_frac": round(v["gbs"] / HBM_PEAK_GBS, 4), "traffic": measured_traffic(W.name, k)}
                  for k, v in kern.items()}

    if args.workload == "B":
        metric = "LS solves/sec at 128^3x60 illum, FP32 vs plain at 1e-4 rel err; p50/p99 ms"
    else:
        metric = f"LS solves/sec at {n}^3x{Q} illum ({W.precision}, tol {W.tol:g}); p50/p99 ms"
    solve_ms = [i["time_ms"] for step_info in r["infos"] for i in step_info]
    assert min(solve_ms) > 0, "every solve reports its device completion time"
    out = {
        "metric": metric,
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * r["total"] / args.steps, 2),
        # per-solve completion time over all timed steps: device clock from the batch's first pass
        # to the step at which that illumination's solve reached its final state
        "p50_ms": round(pct(solve_ms, 50), 2),
        "p99_ms": round(pct(solve_ms, 99), 2),
        "step_p50_ms": round(pct(r["times"], 50), 2),
        "step_p99_ms": round(pct(r["times"], 99), 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if c128 else "c64 fields, f64 reductions",
        "data": data_description(W),
        "config": {"workload": W.name, "n": n, "padded_fft": 2 * n, "illuminations": Q, "group_size": Q, "tol": W.tol,
                   "detector": f"{n}x{n}", "p": W.p, "green_init_ms": round(r["t_init"] * 1e3, 1),
                   "library_load_ms": round(lib_ms, 1)},
        "solve": s,
        "roofline": roof,
        "kernels": per_kernel,
    }
    # illuminations the host oracle solves: four of the benchmark batch, one of the others
    qs = [q for q in (0, 15, 30, 45) if q < Q] if args.workload == "B" else [0]
    gpu_fields = [(q, r["u"][q].cpu().numpy().astype(np.complex128), r["y"][q].cpu().numpy().astype(np.complex128))
                  for q in qs]
    if not args.no_extras and args.workload == "B":
        out["accuracy"] = accuracy_vs_c128(W, r)
    f_np = W.potential()
    release(r)
    if not args.no_extras and args.workload == "B":
        out["configs"] = {"C": config_C(2, 1, 2), "D": config_D(5, 1), "E": config_E()}
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["oracle_check"] = cpu_baseline(W, f_np, gpu_fields)
    print(json.dumps(out), flush=True)
    return 0


def kernel_code_sha(text):
    """First 16 hex digits of the sha256 of kernel source text with its comments, leading and
    trailing blanks and empty lines removed: edits to comments leave it unchanged, edits to code
    do not."""
    import hashlib
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*", "", line).strip() for line in text.splitlines())
    return hashlib.sha256("\n".join(line for line in lines if line).encode()).hexdigest()[:16]


def kernel_sources_text():
    src = os.path.join(ROOT, "paper_1910_13844_amd", "csrc")
    return "".join(open(os.path.join(src, name)).read() for name in ("kernels.hip", "fft.hpp"))


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or
    None when that summary is missing or was taken from different kernel code."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    try:
        sha = kernel_code_sha(kernel_sources_text())
        vals = {}
        for line in open(path):
            if ":" in line and not line.startswith("|"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
        if vals.get("kernel_code_sha256_16") != sha:
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


def cpu_baseline(W, f_np, gpu_fields):
    """The FP64 oracle timed on the host: whole BiCGSTAB solves (all iterations, the workload's
    tolerance) and far fields of the illuminations in gpu_fields [(q, u_q, y_q)], FFTs on all host
    cores.  Its solutions also measure the GPU's: relative L2 of the timed batch's u and y there."""
    from oracle import dft, farfield as ofar
    from oracle import incident, kernel, ops, solver

    n = W.n
    dirs = W.dirs()
    t = time.perf_counter()
    gh = kernel.ghat_m(n, W.p, W.k)
    t_setup = time.perf_counter() - t
    log(f"oracle kernel setup {t_setup:.1f} s")
    t_solve = t_ff = 0.0
    iters, matvecs, eu, ey, rr = [], [], [], [], []
    for q, uq, yq in gpu_fields:
        b = incident.plane_wave(n, W.k, dirs[q])
        t = time.perf_counter()
        uo, info = solver.bicgstab(lambda v: ops.A_apply(gh, f_np, v), b, W.tol)
        t1 = time.perf_counter()
        yo = ofar.farfield_fft(f_np * uo, W.k, W.xg)
        t2 = time.perf_counter()
        t_solve += t1 - t
        t_ff += t2 - t1
        log(f"oracle solve q={q}: {t1 - t:.1f} s ({info.iters} iterations), far field {t2 - t1:.2f} s")
        iters.append(int(info.iters))
        matvecs.append(int(info.matvecs))
        eu.append(rel(uq, uo))
        ey.append(rel(yq, yo))
        rr.append(float(info.relres_true))
    qs = [q for q, _, _ in gpu_fields]
    base = {"value": round(len(qs) / (t_solve + t_ff), 6), "unit": "solves/s", "cores": dft.WORKERS, "kind": "oracle",
            "host": host_description(),
            "sample": (f"{len(qs)} whole FP64 solves of illuminations {qs} of the batch (tol {W.tol:g}; "
                       f"{sum(iters)} iterations, {sum(matvecs)} operator applications in all) = {t_solve:.2f} s "
                       f"+ their far fields {t_ff:.2f} s; FFTs on {dft.WORKERS} threads (scipy.fft), the rest "
                       f"single-threaded numpy; one-time kernel setup {t_setup:.1f} s excluded")}
    check = {"illuminations": qs, "u_rel_l2": eu, "y_rel_l2": ey, "u_rel_l2_max": max(eu), "y_rel_l2_max": max(ey),
             "oracle_iters": iters, "oracle_relres_true": rr, "tol": W.tol,
             "note": "GPU complex64 vs the oracle, both stopped at the workload tolerance"}
    return base, check


if __name__ == "__main__":
    sys.exit(main())
