"""GPU test of ls_forward_farfield_noalloc (the entry point that allocates nothing): through the C ABI
its fields equal those of ls_forward_farfield with a caller workspace, bit for bit, on two calls in
a row on the same device (the second with fewer illuminations and then a smaller grid, so stale
scratch contents from the first call would show), and a grid that does not fit the fixed scratch is
rejected with LS_ERR_WORKSPACE."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_1910_13844_amd import _lib, api, workloads  # noqa: E402

K = workloads.k_of()
DEV = "cuda:0"


def _both(c, Q, seed):
    rd = torch.float64 if c.prec == "c128" else torch.float32
    f = torch.from_numpy(workloads.blob_potential(seed, c.n, dn_max=0.05)).to(DEV, rd)
    dirs = workloads.cone_dirs(Q, 45.0)
    u1, y1, i1 = c.ls_forward_farfield(f, dirs, tol=1e-6)
    u2 = torch.full_like(u1, float("nan"))
    y2 = torch.full_like(y1, float("nan"))
    before = torch.cuda.memory_allocated(DEV)
    i2 = c.ls_forward_farfield_noalloc(f, dirs, u2, y2, tol=1e-6)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(DEV) == before
    print(f"[noalloc] n={c.n} {c.prec} Q={Q}: iterations {[i['iters'] for i in i2]}", flush=True)
    assert [i["status"] for i in i2] == [0] * Q
    assert [(i["iters"], i["matvecs"]) for i in i1] == [(i["iters"], i["matvecs"]) for i in i2]
    assert torch.equal(u1, u2) and torch.equal(y1, y2)


def test_noalloc_equals_workspace_call_twice():
    c64 = api.Context(64, K, p=4, xg=64.0, prec="c64", device=DEV)
    _both(c64, 12, 0)       # 10 illuminations fit the scratch at 64^3: two groups
    _both(c64, 3, 1)        # second call, fewer illuminations
    c32 = api.Context(32, K, p=4, xg=32.0, prec="c128", device=DEV)
    _both(c32, 2, 2)        # then a smaller grid in complex128


def test_noalloc_rejects_a_grid_beyond_the_scratch():
    c = api.Context(144, K, p=4, xg=144.0, prec="c64", device=DEV)
    f = torch.zeros((144,) * 3, dtype=torch.float32, device=DEV)
    u = torch.empty((1, 144, 144, 144), dtype=torch.complex64, device=DEV)
    y = torch.empty((1, 144, 144), dtype=torch.complex64, device=DEV)
    with pytest.raises(_lib.LSError, match="workspace"):
        c.ls_forward_farfield_noalloc(f, [[0.0, 0.0, 1.0]], u, y)
