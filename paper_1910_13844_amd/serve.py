"""Continuous-batching request loop over the slot API (ls_batch_*).

Requests (forward or gradient, any supported grid size, 1..Q illuminations each) arrive over time.
Each illumination solve becomes a job; one slot pool per grid size keeps the Krylov state and the
Green kernels of that size resident on the device.  Between BiCGSTAB steps the loop harvests
finished slots and admits waiting jobs into free slots, so work that arrives while other work is on
the GPU joins the same kernel launches.  A gradient request runs its forward solves, then its far
field and residual, then one adjoint solve per illumination (right-hand side G~^T conj(r)), then the
gradient accumulation.  Each result is the same alone and in a mix: slots never interact (per-slot
reductions in a fixed order).

Admission is by device-memory footprint: the engine keeps a byte ledger (``Ledger``) over one
budget shared by every pool -- the Green kernels and far-field workspaces of each grid size, the slot
pools' workspaces, and every request's own fields (``request_bytes``).  A request's first job is
admitted only when its fields fit in what the budget has left; until then it waits at the head of
its pool's queue (no overtaking), and its bytes return to the budget when it completes.

Engines: ``GpuEngine`` drives libls through ``api``; tests substitute a CPU engine with the same
methods to exercise the scheduler without a GPU.

    python -m paper_1910_13844_amd.serve [--requests 400] [--rate 20] [--grids 64,96,128,192] [--baseline]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import sys
import time
from collections import deque
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    kind: str            # "forward" or "grad"
    n: int
    Q: int
    arrival: float       # seconds from the start of the trace
    seed: int
    theta: float
    # filled by the loop
    done_time: Optional[float] = None
    admitted: bool = False   # its fields hold device memory (first job admitted, not yet complete)
    outputs: dict = dataclasses.field(default_factory=dict)


@dataclasses.dataclass
class Job:
    req: Request
    q: int
    phase: str           # "fwd" or "adj"
    slot: int = -1


def poisson_trace(nreq: int, rate: float, grids: Sequence[int], qmax: int = 60, seed: int = 6,
                  grad_fraction: float = 0.5) -> List[Request]:
    """Poisson arrivals (exponential gaps, mean 1/rate), kind forward/gradient with equal odds,
    grid uniform over `grids`, illuminations uniform over 1..qmax; phantom seed = request id."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(nreq):
        t += rng.exponential(1.0 / rate)
        kind = "grad" if rng.uniform() < grad_fraction else "forward"
        n = int(rng.choice(list(grids)))
        Q = int(rng.integers(1, qmax + 1))
        out.append(Request(i, kind, n, Q, t, seed=i, theta=40.0 if kind == "grad" else 45.0))
    return out


def request_bytes(kind: str, n: int, Q: int, csz: int) -> int:
    """Device bytes a request holds from its first admission to its completion: the total fields u
    (Q N complex) and detector fields y (Q n^2); for gradients also the adjoint solutions w and their
    right-hand sides b (Q N each), the detector residuals (Q n^2), their FP64 sums (2Q) and the
    gradient (N reals).  csz: bytes per complex (8 for complex64)."""
    N, M = n ** 3, n * n
    b = Q * (N + M) * csz
    if kind == "grad":
        b += Q * (2 * N + M) * csz + 2 * Q * 8 + N * (csz // 2)
    return b


class Ledger:
    """A device-memory budget as named charges (thread-safe).  ``charge`` raises MemoryError when a
    charge would exceed the budget; ``try_charge`` reports it instead; ``peak`` is the largest total
    ever charged."""

    def __init__(self, budget: float):
        import threading
        self.budget = int(budget)
        self.charges: Dict[tuple, int] = {}
        self.used = 0
        self.peak = 0
        self._lock = threading.Lock()

    def try_charge(self, key: tuple, nbytes: int) -> bool:
        with self._lock:
            if key in self.charges:
                raise KeyError(f"{key} is already charged")
            if self.used + nbytes > self.budget:
                return False
            self.charges[key] = int(nbytes)
            self.used += int(nbytes)
            self.peak = max(self.peak, self.used)
            return True

    def charge(self, key: tuple, nbytes: int) -> None:
        if not self.try_charge(key, nbytes):
            raise MemoryError(f"{key}: {nbytes} bytes do not fit the device budget ({self.used} of "
                              f"{self.budget} bytes in use)")

    def release(self, key: tuple) -> int:
        with self._lock:
            nbytes = self.charges.pop(key)
            self.used -= nbytes
            return nbytes

    def held(self, kinds: Sequence[str]) -> int:
        """Total of the charges whose key starts with one of `kinds`."""
        with self._lock:
            return sum(v for k, v in self.charges.items() if k[0] in kinds)


class Scheduler:
    """Continuous batching over per-grid-size slot pools.

    engine: object with
      pool_capacity(n) -> int
      reserve(req) -> bool                  -> (optional) charge the request's device footprint;
                                               False: it does not fit now, the request waits
      prepare(req)                          -> per-request device data (potential, directions, data)
      admit(n, slot, job)                   -> start the job's solve in `slot` of pool n
      step(n, iters)                        -> advance every running slot of pool n
      poll(n) -> (states, infos)            -> 0 idle, 1 running, 2 done
      release(n, slot)
      finish_forward(req)                   -> after all forward solves: far field (and, for
                                               gradient requests, residual + adjoint right-hand sides)
      finish_grad(req)                      -> after all adjoint solves: gradient accumulation
    """

    def __init__(self, engine, iters_per_step: int = 2, clock: Callable[[], float] = time.perf_counter,
                 progress: int = 0):
        self.e = engine
        self.progress = progress
        self.iters = iters_per_step
        self.clock = clock
        self.pending: Dict[int, Deque[Job]] = {}
        self.slots: Dict[int, List[Optional[Job]]] = {}
        self.left: Dict[Tuple[int, str], int] = {}
        self.completed: List[Request] = []
        self.solves = 0

    def _pool(self, n):
        if n not in self.slots:
            self.slots[n] = [None] * self.e.pool_capacity(n)
            self.pending[n] = deque()
        return self.slots[n]

    def submit(self, req: Request):
        self._pool(req.n)
        self.left[(req.rid, "fwd")] = req.Q
        for q in range(req.Q):
            self.pending[req.n].append(Job(req, q, "fwd"))

    def _fill(self, n):
        slots = self.slots[n]
        reserve = getattr(self.e, "reserve", None)
        for i, s in enumerate(slots):
            if s is None and self.pending[n]:
                job = self.pending[n][0]
                if not job.req.admitted:
                    # per-request device buffers exist only from the first admission to completion;
                    # a request whose fields do not fit the memory left waits at the head of the queue
                    if reserve is not None and not reserve(job.req):
                        break
                    self.e.prepare(job.req)
                    job.req.admitted = True
                self.pending[n].popleft()
                job.slot = i
                self.e.admit(n, i, job)
                slots[i] = job

    def _harvest(self, n, t0):
        states, infos = self.e.poll(n)
        slots = self.slots[n]
        for i, job in enumerate(slots):
            if job is None or states[i] != 2:
                continue
            self.e.release(n, i)
            slots[i] = None
            self.solves += 1
            req = job.req
            req.outputs.setdefault("info_" + job.phase, {})[job.q] = infos[i]
            key = (req.rid, job.phase)
            self.left[key] -= 1
            if self.left[key] == 0:
                if job.phase == "fwd":
                    self.e.finish_forward(req)
                    if req.kind == "grad":
                        # adjoint solves go ahead of queued work: the request already holds its
                        # fields, and finishing it first bounds both memory and its latency
                        self.left[(req.rid, "adj")] = req.Q
                        self.pending[n].extendleft(Job(req, q, "adj") for q in reversed(range(req.Q)))
                    else:
                        self._complete(req, t0)
                else:
                    self.e.finish_grad(req)
                    self._complete(req, t0)

    def _complete(self, req: Request, t0: float):
        req.done_time = self.clock() - t0
        req.admitted = False
        self.completed.append(req)
        if self.progress and len(self.completed) % self.progress == 0:
            print(f"[serve] {len(self.completed)} requests done at {req.done_time:.1f} s", file=sys.stderr, flush=True)

    def busy(self) -> bool:
        return any(s is not None for pool in self.slots.values() for s in pool) or any(self.pending.values())

    def run(self, trace: Sequence[Request], realtime: bool = True) -> dict:
        trace = sorted(trace, key=lambda r: r.arrival)
        t0 = self.clock()
        nxt = 0
        while nxt < len(trace) or self.busy():
            now = self.clock() - t0
            while nxt < len(trace) and (trace[nxt].arrival <= now or not realtime or not self.busy()):
                if realtime and trace[nxt].arrival > now and not self.busy():
                    # idle: wait for the next arrival
                    time.sleep(max(0.0, trace[nxt].arrival - now))
                self.submit(trace[nxt])
                nxt += 1
                now = self.clock() - t0
            for n in list(self.slots):
                self._fill(n)
                if any(s is not None for s in self.slots[n]):
                    self.e.step(n, self.iters)
                    self._harvest(n, t0)
        total = self.clock() - t0
        return summarize(self.completed, total, self.solves)


class ConcurrentScheduler(Scheduler):
    """The same continuous batching with one host thread per slot pool.  Each pool's thread fills,
    steps and harvests its pool inside ``engine.stream_context(n)`` (for the GPU engine, a stream of
    its own), so the pools of different grid sizes run on the device at the same time and one
    pool's host work (admissions, far fields of finished requests) overlaps the others' kernels.
    All scheduler state is guarded by one lock; the engine's step runs outside it."""

    def run(self, trace: Sequence[Request], realtime: bool = True) -> dict:
        import contextlib
        import threading

        trace = sorted(trace, key=lambda r: r.arrival)
        t0 = self.clock()
        cv = threading.Condition()
        state = {"closed": False, "error": None}
        workers: Dict[int, threading.Thread] = {}
        stream_context = getattr(self.e, "stream_context", None)

        def pool_busy(n):
            return any(s is not None for s in self.slots[n]) or bool(self.pending[n])

        def worker(n):
            try:
                with (stream_context(n) if stream_context else contextlib.nullcontext()):
                    while True:
                        with cv:
                            while True:
                                if state["error"] is not None or (state["closed"] and not pool_busy(n)):
                                    return
                                if pool_busy(n):
                                    self._fill(n)
                                    if any(s is not None for s in self.slots[n]):
                                        break
                                # idle, or the queue's head waits for device memory that another
                                # pool's completions will return (they notify)
                                cv.wait(0.05)
                        self.e.step(n, self.iters)
                        with cv:
                            self._harvest(n, t0)
                            cv.notify_all()
            except BaseException as exc:  # reported by run() after the threads have stopped
                with cv:
                    state["error"] = exc
                    cv.notify_all()

        for req in trace:
            now = self.clock() - t0
            if realtime and req.arrival > now:
                time.sleep(req.arrival - now)
            with cv:
                if state["error"] is not None:
                    break
                self.submit(req)
                if req.n not in workers:
                    workers[req.n] = threading.Thread(target=worker, args=(req.n,), daemon=True)
                    workers[req.n].start()
                cv.notify_all()
        with cv:
            state["closed"] = True
            cv.notify_all()
        for w in workers.values():
            w.join()
        if state["error"] is not None:
            raise state["error"]
        if hasattr(self.e, "synchronize"):
            self.e.synchronize()
        total = self.clock() - t0
        return summarize(self.completed, total, self.solves)


def summarize(done: Sequence[Request], total: float, solves: int) -> dict:
    lat = [r.done_time - r.arrival for r in done]
    return {"requests": len(done), "solves": solves, "seconds": total,
            "solves_per_s": solves / total if total > 0 else float("nan"),
            "p50_ms": 1e3 * float(np.percentile(lat, 50)) if lat else None,
            "p99_ms": 1e3 * float(np.percentile(lat, 99)) if lat else None}


# ---------------------------------------------------------------------------------------------
class GpuEngine:
    """Scheduler engine backed by libls on one GPU, with every device buffer it allocates charged to
    one budget (``ledger``): per grid size the Green kernels and a far-field workspace for
    ``ff_group`` illuminations, the slot pool's workspace (pools share ``pool_fraction`` of the budget
    evenly over the grid sizes served, at most ``max_slots`` slots each), and each admitted
    request's fields (``request_bytes``).  Request inputs (potentials, directions, measurements)
    are preloaded before the trace starts and are not part of the budget."""

    def __init__(self, hbm_budget_gb: float = 120.0, tol: float = 1e-5, maxit: int = 500, prec: str = "c64",
                 device: str = "cuda:0", max_slots: int = 64, inputs: Optional[dict] = None,
                 grids: Optional[Sequence[int]] = None, pool_fraction: float = 0.5, ff_group: int = 8):
        import torch

        from . import _lib, api, workloads

        self.torch, self.api, self.wl, self._lib = torch, api, workloads, _lib
        self.tol, self.maxit, self.prec, self.device = tol, maxit, prec, device
        self.ledger = Ledger(hbm_budget_gb * 1e9)
        self.max_slots = max_slots
        self.pool_fraction = pool_fraction
        self.ff_group = ff_group
        self.grids: List[int] = sorted(set(grids)) if grids else []
        self.csz = 8 if prec == "c64" else 16
        self.ctx: Dict[int, "api.Context"] = {}
        self.ffws: Dict[int, "torch.Tensor"] = {}
        self.pool: Dict[int, "api.Batch"] = {}
        self.cap: Dict[int, int] = {}
        self.data: Dict[int, dict] = {}
        self.streams: Dict[int, "torch.cuda.Stream"] = {}
        # request inputs (potential, directions, measurements) keyed by request id; may be shared
        # between engines on the same device so that a trace is generated once
        self.inputs: Dict[int, dict] = {} if inputs is None else inputs

    def stream_context(self, n):
        """Context manager that makes pool n's own stream current (default priority)."""
        if n not in self.streams:
            self.streams[n] = self.torch.cuda.Stream(device=self.device)
        return self.torch.cuda.stream(self.streams[n])

    def synchronize(self):
        self.torch.cuda.synchronize(self.device)

    def _ctx(self, n):
        if n not in self.ctx:
            c = self.api.Context(n, self.wl.k_of(), p=4, xg=float(n), prec=self.prec, device=self.device)
            self.ledger.charge(("ctx", n), c.kbuf.numel())
            nb = c.workspace_bytes(self.ff_group, self._lib.LS_OP_FARFIELD)
            self.ledger.charge(("ws", n), nb)
            self.ffws[n] = self.torch.empty(nb, dtype=self.torch.uint8, device=self.device)
            self.ctx[n] = c
        return self.ctx[n]

    def pool_capacity(self, n):
        if n in self.cap:
            return self.cap[n]
        if n not in self.grids:
            self.grids.append(n)
        c = self._ctx(n)
        per_slot = c.workspace_bytes(2, self._lib.LS_OP_FORWARD) - c.workspace_bytes(1, self._lib.LS_OP_FORWARD)
        share = self.pool_fraction * self.ledger.budget / max(1, len(self.grids))
        cap = int(min(self.max_slots, share // max(per_slot, 1)))
        if cap < 1:
            raise MemoryError(f"grid {n}: one slot ({per_slot} bytes) exceeds the pool share of the budget")
        pool = self.api.Batch(c, cap, tol=self.tol, maxit=self.maxit)
        self.ledger.charge(("pool", n), pool.ws.numel())
        self.pool[n], self.cap[n] = pool, cap
        return cap

    def reserve(self, req: Request) -> bool:
        nbytes = request_bytes(req.kind, req.n, req.Q, self.csz)
        free_at_best = self.ledger.budget - self.ledger.held(("ctx", "ws", "pool"))
        if nbytes > free_at_best:
            raise MemoryError(f"request {req.rid}: {nbytes} bytes can never fit the budget ({free_at_best} bytes "
                              "left beside the kernels and slot pools)")
        return self.ledger.try_charge(("req", req.rid), nbytes)

    def memory_report(self) -> dict:
        """Ledger totals (what the loop charged: peak and the fixed part), and the allocator's view: the
        bytes allocated once the inputs were preloaded (fixed part + inputs) and the peak while serving."""
        return {"budget_bytes": self.ledger.budget, "peak_bytes": self.ledger.peak,
                "fixed_bytes": self.ledger.held(("ctx", "ws", "pool")),
                "allocated_after_preload_bytes": getattr(self, "preloaded_bytes", None),
                "allocated_peak_while_serving_bytes": int(self.torch.cuda.max_memory_allocated(self.device))}

    def preload(self, trace: Sequence[Request], workers: int = 8):
        """Generate every request's inputs before the trace starts (not part of the served work):
        the potential, the illumination directions and, for gradient requests, synthetic measurements
        of a perturbed phantom.  Phantoms are generated on `workers` host threads.  Also builds the
        kernels and slot pools of every grid size in the trace, so the budget's fixed part is known
        before the first admission."""
        import concurrent.futures as cf

        torch = self.torch
        for n in sorted(set(r.n for r in trace)):
            if n not in self.grids:
                self.grids.append(n)
        for n in sorted(set(r.n for r in trace)):
            self.pool_capacity(n)
        todo = [r for r in trace if r.rid not in self.inputs]

        def phantoms(req):
            f = self.wl.blob_potential(req.seed, req.n, dn_max=0.05)
            pert = None
            if req.kind == "grad":
                pert = self.wl.blob_potential(req.seed + 100000, req.n, nblobs=5, sigma_range=(2.0, 5.0),
                                              dn_max=0.01)
            return f, pert

        with cf.ThreadPoolExecutor(max_workers=workers) as ex:
            for req, (f, pert) in zip(todo, ex.map(phantoms, todo)):
                c = self._ctx(req.n)
                d = {"f": torch.from_numpy(f).to(self.device, c.rdtype), "dirs": self.wl.cone_dirs(req.Q, req.theta)}
                if pert is not None:
                    ft = torch.from_numpy(f + pert).to(self.device, c.rdtype)
                    ut, _ = c.ls_forward(ft, d["dirs"], tol=self.tol)
                    d["y_meas"] = c.ls_farfield(ft, ut)
                    del ut, ft
                self.inputs[req.rid] = d
        for c in self.ctx.values():   # scratch of the measurement solves
            c._ws.clear()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        # device memory held before serving starts: the kernels, far-field workspaces and slot pools
        # (charged to the ledger) and the preloaded request inputs (not charged)
        self.preloaded_bytes = int(torch.cuda.memory_allocated(self.device))
        torch.cuda.reset_peak_memory_stats(self.device)

    def prepare(self, req: Request):
        c = self._ctx(req.n)
        d = dict(self.inputs[req.rid])
        d["u"] = self.torch.empty((req.Q, req.n, req.n, req.n), dtype=c.cdtype, device=self.device)
        if req.kind == "grad":
            d["w"] = self.torch.empty_like(d["u"])
        self.data[req.rid] = d

    def admit(self, n, slot, job: Job):
        d = self.data[job.req.rid]
        if job.phase == "fwd":
            self.pool[n].ls_batch_admit(slot, d["f"], d["u"][job.q], direction=d["dirs"][job.q])
        else:
            self.pool[n].ls_batch_admit(slot, d["f"], d["w"][job.q], rhs=d["b"][job.q])

    def step(self, n, iters):
        self.pool[n].ls_batch_step(iters)

    def poll(self, n):
        return self.pool[n].ls_batch_poll()

    def release(self, n, slot):
        self.pool[n].ls_batch_release(slot)

    def _done(self, req: Request):
        self.data.pop(req.rid, None)
        self.torch.cuda.current_stream().synchronize()   # the request is complete when its outputs are
        self.ledger.release(("req", req.rid))

    def finish_forward(self, req: Request):
        c = self.ctx[req.n]
        d = self.data[req.rid]
        ws = self.ffws[req.n]
        d["y"] = c.ls_farfield(d["f"], d["u"], ws=ws)
        if req.kind == "grad":
            r, d["stats"], loss = c.ls_residual(d["y"], d["y_meas"])
            d["loss"] = float(loss)
            d["b"] = c.ls_farfield_adj(r, conj=True, ws=ws)
        else:
            req.outputs["y"] = d["y"]
            self._done(req)

    def finish_grad(self, req: Request):
        d = self.data[req.rid]
        c = self.ctx[req.n]
        g = self.torch.empty((req.n,) * 3, dtype=c.rdtype, device=self.device)
        req.outputs["grad"] = c.ls_grad_accumulate(d["u"], d["w"], g, stats=d["stats"])
        req.outputs["loss"] = d["loss"]
        self._done(req)


def one_at_a_time(engine_factory, trace: Sequence[Request], progress: int = 50) -> dict:
    """Baseline: requests served in arrival order, each illumination solved alone (Q = 1 calls)."""
    import torch

    e = engine_factory()
    e.preload(trace)
    t0 = time.perf_counter()
    solves = 0
    done = []
    for req in sorted(trace, key=lambda r: r.arrival):
        now = time.perf_counter() - t0
        if req.arrival > now:
            time.sleep(req.arrival - now)
        if not e.reserve(req):
            raise MemoryError(f"request {req.rid} does not fit the budget even alone")
        e.prepare(req)
        c = e._ctx(req.n)
        d = e.data[req.rid]
        for q in range(req.Q):
            c.ls_forward(d["f"], d["dirs"][q:q + 1], tol=e.tol, u=d["u"][q:q + 1])
            solves += 1
        if req.kind == "grad":
            e.finish_forward(req)
            bt = e.api.Batch(c, 1, tol=e.tol, maxit=e.maxit)
            for q in range(req.Q):
                # adjoint solve for one illumination (stored right-hand side) through a one-slot pool
                bt.ls_batch_admit(0, d["f"], d["w"][q], rhs=d["b"][q])
                while bt.ls_batch_poll()[0][0] != 2:
                    bt.ls_batch_step(2)
                bt.ls_batch_release(0)
                solves += 1
            e.finish_grad(req)
        else:
            e.finish_forward(req)
        req.done_time = time.perf_counter() - t0
        done.append(req)
        if progress and len(done) % progress == 0:
            print(f"[serve] one-at-a-time: {len(done)} requests done at {req.done_time:.1f} s", file=sys.stderr,
                  flush=True)
    torch.cuda.synchronize()
    return summarize(done, time.perf_counter() - t0, solves)


def _max_rel_diff(a: Sequence[Request], b: Sequence[Request]) -> float:
    """Largest relative difference between the outputs (detector fields or gradients) that two runs
    produced for the same requests."""
    ob = {r.rid: r.outputs for r in b}
    worst = 0.0
    for r in a:
        for key in ("y", "grad"):
            x, y = r.outputs.get(key), ob.get(r.rid, {}).get(key)
            if x is not None and y is not None:
                d = float((x - y).abs().pow(2).sum().sqrt() / y.abs().pow(2).sum().sqrt().clamp_min(1e-300))
                worst = max(worst, d)
    return worst


def benchmark(requests: int = 400, rate: float = 20.0, grids: Sequence[int] = (64, 96, 128, 192), qmax: int = 60,
              budget_gb: float = 120.0, baseline: bool = False, single_thread: bool = False,
              progress: int = 50) -> dict:
    """Serves a seeded Poisson trace with continuous batching on the GPU and, with `baseline`, the
    same requests one illumination at a time; returns the throughput and latency summaries, the
    memory report and the largest difference between the two runs' results."""
    import torch

    grids = list(grids)
    mk = lambda: poisson_trace(requests, rate, grids, qmax)  # noqa: E731
    inputs: dict = {}
    eng = GpuEngine(hbm_budget_gb=budget_gb, inputs=inputs)
    trace = mk()
    t = time.perf_counter()
    eng.preload(trace)
    print(f"[serve] inputs for {len(trace)} requests ready in {time.perf_counter() - t:.1f} s", file=sys.stderr,
          flush=True)
    sched = (Scheduler if single_thread else ConcurrentScheduler)(eng, progress=progress)
    res = {"continuous": sched.run(trace)}
    torch.cuda.synchronize()
    res["continuous"]["memory"] = eng.memory_report()
    print(f"[serve] continuous: {res['continuous']}", file=sys.stderr, flush=True)
    del sched, eng
    torch.cuda.empty_cache()
    if baseline:
        trace_b = mk()
        res["one_at_a_time"] = one_at_a_time(lambda: GpuEngine(hbm_budget_gb=budget_gb, inputs=inputs), trace_b,
                                             progress=progress)
        res["alone_vs_mix_max_rel"] = _max_rel_diff(trace, trace_b)
        torch.cuda.empty_cache()
    nsolve = sum(r.Q * (2 if r.kind == "grad" else 1) for r in trace)
    res["config"] = {"requests": requests, "rate": rate, "grids": grids, "qmax": qmax,
                     "scheduler": "single thread" if single_thread else "one thread and stream per pool",
                     "solves_in_trace": nsolve, "trace_seconds": max(r.arrival for r in trace)}
    return res


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=400)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--grids", default="64,96,128,192")
    ap.add_argument("--qmax", type=int, default=60)
    ap.add_argument("--budget-gb", type=float, default=120.0)
    ap.add_argument("--baseline", action="store_true", help="also run the one-solve-at-a-time baseline")
    ap.add_argument("--single-thread", action="store_true",
                    help="step the slot pools one after the other from one host thread")
    args = ap.parse_args(argv)
    res = benchmark(args.requests, args.rate, [int(g) for g in args.grids.split(",")], args.qmax, args.budget_gb,
                    args.baseline, args.single_thread)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
