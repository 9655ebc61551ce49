"""Edge cases through the C ABI: batches larger than the workspace (processed in groups), a single
illumination, argument errors, bitwise determinism of repeated calls, and the device-recorded
completion time of each solve.

A group's results must not depend on how the batch is split: the slots never interact and every
reduction runs in a fixed order, so solutions, detector fields and gradients computed with a
workspace for two illuminations equal those computed with room for all of them, bit for bit.
"""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1910_13844_amd import _lib, api, workloads  # noqa: E402

K = workloads.k_of()
DEV = "cuda:0"


@pytest.fixture(scope="module")
def c():
    return api.Context(32, K, p=4, xg=32.0, prec="c64", device=DEV)


def test_forward_split_into_groups_is_bitwise_identical(c):
    n, Q = 32, 5
    f = torch.from_numpy(workloads.blob_potential(0, n, dn_max=0.05).astype(np.float32)).to(DEV)
    dirs = workloads.cone_dirs(Q, 45.0)
    u_full, i_full = c.ls_forward(f, dirs, tol=1e-6)
    per2 = c.workspace_bytes(2, _lib.LS_OP_FORWARD)
    ws_small = torch.empty(per2, dtype=torch.uint8, device=DEV)      # room for 2 of the 5
    u_grp, i_grp = c.ls_forward(f, dirs, tol=1e-6, ws=ws_small)
    assert torch.equal(u_full, u_grp)
    assert [i["iters"] for i in i_full] == [i["iters"] for i in i_grp]
    y_full = c.ls_farfield(f, u_full)
    y_grp = c.ls_farfield(f, u_full, ws=torch.empty(c.workspace_bytes(2, _lib.LS_OP_FARFIELD), dtype=torch.uint8,
                                                    device=DEV))
    assert torch.equal(y_full, y_grp)
    # and the same again: repeated calls are deterministic
    u_again, _ = c.ls_forward(f, dirs, tol=1e-6)
    assert torch.equal(u_full, u_again)


def test_gradient_split_into_groups_is_bitwise_identical(c):
    n, Q = 32, 4
    f0, ft = workloads.perturbed_potential(n)
    f0t = torch.from_numpy(f0.astype(np.float32)).to(DEV)
    dirs = workloads.cone_dirs(Q, 40.0)
    u, _ = c.ls_forward(torch.from_numpy(ft.astype(np.float32)).to(DEV), dirs, tol=1e-6)
    y = c.ls_farfield(torch.from_numpy(ft.astype(np.float32)).to(DEV), u)
    l1, g1, _ = c.ls_grad(f0t, dirs, y, tol=1e-6)
    ws_small = torch.empty(c.workspace_bytes(1, _lib.LS_OP_GRAD), dtype=torch.uint8, device=DEV)
    l2, g2, _ = c.ls_grad(f0t, dirs, y, tol=1e-6, ws=ws_small)
    # the gradient accumulates group by group in FP64 and is rounded once: same bits either way
    assert torch.equal(g1, g2) and l1 == l2


def test_single_illumination_and_errors(c):
    n = 32
    f = torch.zeros((n, n, n), dtype=torch.float32, device=DEV)
    u, info = c.ls_forward(f, [[0.0, 0.0, 1.0]], tol=1e-6)
    assert u.shape == (1, n, n, n) and info[0]["status"] == 0 and info[0]["iters"] <= 1
    uin = np.exp(1j * K * (np.arange(n) - n // 2 + 1))[:, None, None] * np.ones((1, n, n))   # f = 0: u = u_in
    assert np.abs(u[0].cpu().numpy() - uin).max() < 1e-5
    with pytest.raises(_lib.LSError):
        c.ls_forward(f, np.zeros((0, 3)), tol=1e-6)                           # Q = 0
    with pytest.raises(_lib.LSError):
        c.ls_forward(f, [[0.0, 0.0, 1.0]], tol=-1.0)                          # bad tolerance
    tiny = torch.empty(16, dtype=torch.uint8, device=DEV)
    with pytest.raises(_lib.LSError):
        c.ls_forward(f, [[0.0, 0.0, 1.0]], tol=1e-6, ws=tiny)                 # workspace too small
    with pytest.raises(ValueError):
        c.ls_forward(torch.zeros((n, n, n - 1), dtype=torch.float32, device=DEV), [[0, 0, 1]])


def test_device_completion_times(c):
    n, Q = 32, 6
    f = torch.from_numpy(workloads.blob_potential(1, n, dn_max=0.1).astype(np.float32)).to(DEV)
    dirs = workloads.cone_dirs(Q, 45.0)
    runs = {}
    for tol in (1e-5, 1e-6):
        c.ls_forward(f, dirs, tol=tol)                     # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = c.ls_forward(f, dirs, tol=tol)
        wall = (time.perf_counter() - t0) * 1e3
        ts = [i["time_ms"] for i in info]
        its = [i["iters"] for i in info]
        print(f"[times] tol {tol:g}: iterations {its}, restarts {[i['restarts'] for i in info]}, device ms "
              f"{[round(t, 3) for t in ts]}, call {wall:.3f} ms", flush=True)
        assert all(0 < t <= wall for t in ts)
        # the slots advance in lockstep and the true-residual check runs after every second iteration,
        # so of two slots that never restarted, one whose last iteration fell in a later pair of
        # iterations finished at a later check (a restart shifts a slot's count against the pairs)
        for a in range(Q):
            for b in range(Q):
                if info[a]["restarts"] == 0 and info[b]["restarts"] == 0 and (its[b] + 1) // 2 > (its[a] + 1) // 2:
                    assert ts[b] > ts[a]
        runs[tol] = (its, ts)
    # the tighter tolerance needs more iterations of the same batch and finishes later
    assert min(runs[1e-6][0]) > max(runs[1e-5][0]) and min(runs[1e-6][1]) > max(runs[1e-5][1])
    # gradient calls report both solves of every view
    f0, ft = workloads.perturbed_potential(n)
    y = c.ls_farfield(torch.from_numpy(ft.astype(np.float32)).to(DEV),
                      c.ls_forward(torch.from_numpy(ft.astype(np.float32)).to(DEV), dirs, tol=1e-6)[0])
    _, _, ginfo = c.ls_grad(torch.from_numpy(f0.astype(np.float32)).to(DEV), dirs, y, tol=1e-6)
    assert len(ginfo) == 2 * Q and all(i["time_ms"] > 0 for i in ginfo)


def test_one_context_two_streams_two_threads(c):
    # the context is immutable after ls_green_init: two host threads may drive it on two streams
    # (each with its own workspace) at once, with the same results as one after the other
    import threading
    n, Q = 32, 4
    dirs = workloads.cone_dirs(Q, 45.0)
    fs = [torch.from_numpy(workloads.blob_potential(s, n, dn_max=0.05).astype(np.float32)).to(DEV) for s in (2, 3)]
    refs = [c.ls_forward(f, dirs, tol=1e-6)[0] for f in fs]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    wss = [torch.empty(c.workspace_bytes(Q, _lib.LS_OP_FORWARD), dtype=torch.uint8, device=DEV) for _ in fs]
    outs = [torch.empty_like(r) for r in refs]
    torch.cuda.synchronize()
    errors = []

    def run(i):
        try:
            for _ in range(3):
                c.ls_forward(fs[i], dirs, tol=1e-6, u=outs[i], ws=wss[i], stream=streams[i])
        except Exception as e:  # reported after join
            errors.append(e)

    th = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=120)
    torch.cuda.synchronize()
    assert not errors and not any(t.is_alive() for t in th)
    assert torch.equal(outs[0], refs[0]) and torch.equal(outs[1], refs[1])


def test_binding_rejects_mis_sized_buffers(c):
    # the library sees only pointers: the binding checks every caller buffer before the call, so a
    # wrong size is a ValueError and never an access outside an allocation
    n = 32
    f = torch.zeros((n, n, n), dtype=torch.float32, device=DEV)
    dirs = workloads.cone_dirs(3, 30.0)
    with pytest.raises(ValueError):
        c.ls_forward(f, dirs, u=torch.empty((2, n, n, n), dtype=torch.complex64, device=DEV))   # Q = 3
    u, _ = c.ls_forward(f, dirs, tol=1e-6)
    with pytest.raises(ValueError):
        c.ls_vjp(f, u, torch.zeros((2, n, n), dtype=torch.complex64, device=DEV))
    with pytest.raises(ValueError):
        c.ls_grad(f, dirs, torch.zeros((3, n, n), dtype=torch.complex128, device=DEV))          # dtype
    with pytest.raises(ValueError):
        c.ls_residual(torch.zeros((3, n, n), dtype=torch.complex64, device=DEV),
                      torch.zeros((2, n, n), dtype=torch.complex64, device=DEV))
    with pytest.raises(ValueError):
        c.ls_grad_accumulate(u, u[:2].contiguous(), torch.zeros((n, n, n), dtype=torch.float32, device=DEV))
    b = api.Batch(c, 2)
    with pytest.raises(ValueError):
        b.ls_batch_admit(0, f, torch.empty((n, n, n - 1), dtype=torch.complex64, device=DEV), direction=[0, 0, 1])
