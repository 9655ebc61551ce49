"""CPU tests of the continuous-batching scheduler with a fake engine (no GPU): admission into free
slots as they open, FIFO order, the two phases of gradient requests, capacity limits, latency
accounting.  The fake engine finishes a job after a fixed number of iterations derived from its
request, which is all the scheduler observes of a solve."""
import numpy as np
import pytest

from paper_1910_13844_amd import serve


class FakeEngine:
    def __init__(self, capacity=3):
        self.capacity = capacity
        self.running = {}      # (n, slot) -> [job, iterations left]
        self.log = []
        self.t = 0.0
        self.max_busy = {}

    def clock(self):
        return self.t

    def pool_capacity(self, n):
        return self.capacity

    def prepare(self, req):
        self.log.append(("prepare", req.rid))

    def admit(self, n, slot, job):
        assert (n, slot) not in self.running
        need = 1 + (job.req.rid + job.q) % 4 + (2 if job.phase == "adj" else 0)
        self.running[(n, slot)] = [job, need]
        self.log.append(("admit", job.req.rid, job.q, job.phase, slot))
        busy = sum(1 for (m, _) in self.running if m == n)
        self.max_busy[n] = max(self.max_busy.get(n, 0), busy)

    def step(self, n, iters):
        self.t += 0.01
        for key, v in self.running.items():
            if key[0] == n and v[1] > 0:
                v[1] = max(0, v[1] - iters)

    def poll(self, n):
        st = [0] * self.capacity
        infos = [{"status": 0}] * self.capacity
        for (m, s), v in self.running.items():
            if m == n:
                st[s] = 2 if v[1] == 0 else 1
        return st, infos

    def release(self, n, slot):
        del self.running[(n, slot)]

    def finish_forward(self, req):
        self.log.append(("ffwd", req.rid))

    def finish_grad(self, req):
        self.log.append(("fgrad", req.rid))


def test_all_requests_complete_with_capacity_respected():
    trace = serve.poisson_trace(12, 50.0, [16, 32], qmax=5, seed=1)
    eng = FakeEngine(capacity=3)
    sch = serve.Scheduler(eng, iters_per_step=1, clock=eng.clock)
    res = sch.run(trace, realtime=False)
    assert res["requests"] == 12
    assert res["solves"] == sum(r.Q * (2 if r.kind == "grad" else 1) for r in trace)
    assert all(v <= 3 for v in eng.max_busy.values())
    assert not eng.running
    # gradient requests: forward finish, then adjoint jobs, then gradient finish
    for r in trace:
        ev = [e for e in eng.log if len(e) >= 2 and e[1] == r.rid]
        names = [e[0] for e in ev]
        assert names.count("ffwd") == 1
        if r.kind == "grad":
            assert names.count("fgrad") == 1
            first_adj = min(i for i, e in enumerate(ev) if e[0] == "admit" and e[3] == "adj")
            assert names.index("ffwd") < first_adj < names.index("fgrad")
        else:
            assert "fgrad" not in names


def test_jobs_admitted_in_fifo_order_per_pool():
    trace = [serve.Request(i, "forward", 16, 2, 0.0, i, 45.0) for i in range(4)]
    eng = FakeEngine(capacity=2)
    serve.Scheduler(eng, iters_per_step=1, clock=eng.clock).run(trace, realtime=False)
    adm = [(e[1], e[2]) for e in eng.log if e[0] == "admit"]
    assert adm == [(r, q) for r in range(4) for q in range(2)]


def test_slots_are_refilled_while_others_run():
    # a long job keeps one slot busy while short jobs flow through the other
    trace = [serve.Request(0, "forward", 16, 1, 0.0, 0, 45.0), serve.Request(1, "forward", 16, 3, 0.0, 1, 45.0)]
    eng = FakeEngine(capacity=2)
    eng_admit = eng.admit

    def admit(n, slot, job):
        eng_admit(n, slot, job)
        if job.req.rid == 0:
            eng.running[(n, slot)][1] = 50
    eng.admit = admit
    sch = serve.Scheduler(eng, iters_per_step=1, clock=eng.clock)
    res = sch.run(trace, realtime=False)
    done = {r.rid: r.done_time for r in sch.completed}
    assert done[1] < done[0]
    assert res["requests"] == 2


def test_latency_summary():
    reqs = [serve.Request(i, "forward", 16, 1, float(i), i, 45.0, done_time=float(i) + 0.5) for i in range(10)]
    s = serve.summarize(reqs, 10.0, 10)
    assert abs(s["p50_ms"] - 500.0) < 1e-9 and s["solves_per_s"] == 1.0


class LockedFakeEngine(FakeEngine):
    """FakeEngine safe to call from several threads (the concurrent scheduler steps pools in parallel)."""

    def __init__(self, capacity=3):
        import threading
        super().__init__(capacity)
        self._lock = threading.Lock()

    def admit(self, n, slot, job):
        with self._lock:
            super().admit(n, slot, job)

    def step(self, n, iters):
        with self._lock:
            super().step(n, iters)

    def poll(self, n):
        with self._lock:
            return super().poll(n)

    def release(self, n, slot):
        with self._lock:
            super().release(n, slot)


def test_concurrent_scheduler_completes_the_same_work():
    # one thread per pool: every request completes, capacities hold, and each request sees its
    # phases in order, as with the single-threaded loop
    trace = serve.poisson_trace(16, 50.0, [16, 32, 48], qmax=5, seed=3)
    eng = LockedFakeEngine(capacity=3)
    sch = serve.ConcurrentScheduler(eng, iters_per_step=1, clock=eng.clock)
    res = sch.run(trace, realtime=False)
    assert res["requests"] == 16
    assert res["solves"] == sum(r.Q * (2 if r.kind == "grad" else 1) for r in trace)
    assert all(v <= 3 for v in eng.max_busy.values())
    assert not eng.running
    for r in trace:
        names = [e[0] for e in eng.log if len(e) >= 2 and e[1] == r.rid]
        assert names.count("ffwd") == 1 and names.count("fgrad") == (1 if r.kind == "grad" else 0)


class BudgetFakeEngine(FakeEngine):
    """FakeEngine whose requests hold device bytes (serve.request_bytes, complex64) from their first
    admission to completion, charged to a serve.Ledger the way the GPU engine charges them."""

    def __init__(self, capacity, budget):
        super().__init__(capacity)
        self.ledger = serve.Ledger(budget)
        self.live = set()
        self.max_live = 0

    def reserve(self, req):
        nbytes = serve.request_bytes(req.kind, req.n, req.Q, 8)
        if nbytes > self.ledger.budget:
            raise MemoryError(req.rid)
        ok = self.ledger.try_charge(("req", req.rid), nbytes)
        self.log.append(("reserve", req.rid, ok))
        return ok

    def prepare(self, req):
        super().prepare(req)
        self.live.add(req.rid)
        self.max_live = max(self.max_live, len(self.live))

    def _done(self, req):
        self.live.discard(req.rid)
        self.ledger.release(("req", req.rid))

    def finish_forward(self, req):
        super().finish_forward(req)
        if req.kind == "forward":
            self._done(req)

    def finish_grad(self, req):
        super().finish_grad(req)
        self._done(req)


def test_request_bytes_counts_every_request_owned_field():
    n, Q, c = 64, 3, 8
    N, M = n ** 3, n * n
    assert serve.request_bytes("forward", n, Q, c) == Q * (N + M) * c                      # u, y
    assert serve.request_bytes("grad", n, Q, c) == (Q * (3 * N + 2 * M) * c + 2 * Q * 8   # u w b, y r, stats
                                                    + N * 4)                                # gradient


@pytest.mark.parametrize("sched", ["single", "concurrent"])
def test_admission_by_footprint_never_exceeds_the_budget(sched):
    # a burst of requests (64^3 gradients, 2 illuminations: 13 MB each in complex64) into a pool of
    # 8 slots and a budget that holds two of them: the ledger never passes the budget, at most two
    # requests hold fields at once, the others wait (reserve refused) instead of allocating although
    # slots are free, and all complete
    per = serve.request_bytes("grad", 64, 2, 8)
    trace = [serve.Request(i, "grad", 64, 2, 0.0, i, 40.0) for i in range(6)]
    eng = (BudgetLockedFakeEngine if sched == "concurrent" else BudgetFakeEngine)(capacity=8, budget=2.5 * per)
    cls = serve.ConcurrentScheduler if sched == "concurrent" else serve.Scheduler
    res = cls(eng, iters_per_step=1, clock=eng.clock).run(trace, realtime=False)
    assert res["requests"] == 6
    assert eng.ledger.peak <= eng.ledger.budget and eng.ledger.used == 0
    assert eng.max_live == 2
    assert any(e[0] == "reserve" and not e[2] for e in eng.log)
    # a refused request is admitted later, in arrival order
    first = [e[1] for e in eng.log if e[0] == "prepare"]
    assert first == sorted(first)


def test_request_that_can_never_fit_is_an_error():
    trace = [serve.Request(0, "grad", 64, 40, 0.0, 0, 40.0)]
    eng = BudgetFakeEngine(capacity=4, budget=1e6)
    with pytest.raises(MemoryError):
        serve.Scheduler(eng, iters_per_step=1, clock=eng.clock).run(trace, realtime=False)


def test_ledger_charges():
    led = serve.Ledger(100)
    led.charge(("pool", 1), 60)
    assert not led.try_charge(("req", 1), 50) and led.used == 60
    assert led.try_charge(("req", 2), 40) and led.used == 100 and led.peak == 100
    with pytest.raises(MemoryError):
        led.charge(("req", 3), 1)
    assert led.release(("req", 2)) == 40 and led.used == 60 and led.held(("pool",)) == 60


class BudgetLockedFakeEngine(BudgetFakeEngine, LockedFakeEngine):
    """Thread-safe BudgetFakeEngine for the concurrent scheduler."""

    def __init__(self, capacity, budget):
        LockedFakeEngine.__init__(self, capacity)
        self.ledger = serve.Ledger(budget)
        self.live = set()
        self.max_live = 0
