"""The paper's bead experiment (Fig. 2): a plane wave (lambda0 = 532 nm) through a bead of diameter
3 lambda0 and index 1.4388 in water (1.3388), voxel h = lambda0 / 16, p = 4; total field of the
Lippmann-Schwinger model (GPU) and of the Born model (GPU operator) against the Mie series
(oracle.mie) on the central x-z plane.

The paper shows the fields as images only (no numbers), so this is a physics check with its own
bars: the LS error is below a percent or so (voxelised sphere) and far below the Born error.  Run
at the paper's n = 144 (a 9 lambda0 box, transform lengths 144 and 288) and at n = 128.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import mie  # noqa: E402
from paper_1910_13844_amd import api, workloads  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("n", [144, 128])
def test_bead_ls_vs_born_vs_mie(n):
    eta_b, eta_s, h_over_lambda = 1.3388, 1.4388, 1.0 / 16.0
    radius = 1.5 / h_over_lambda                          # 3 lambda0 diameter, in voxels
    k = workloads.k_of(h_over_lambda, eta_b)
    f = workloads.sphere_potential(n, radius, eta_s, eta_b=eta_b, h_over_lambda=h_over_lambda)
    c = api.Context(n, k, p=4, xg=float(n), prec="c128", device=DEV)
    ft = torch.from_numpy(f).to(DEV)
    u, info = c.ls_forward(ft, [[0.0, 0.0, 1.0]], tol=1e-10, maxit=2000)
    assert info[0]["status"] == 0
    uin = torch.from_numpy(np.exp(1j * k * (np.arange(n) - n // 2 + 1))[:, None, None]
                           * np.ones((1, n, n))).to(DEV)[None].contiguous()
    born = 2 * uin - c.ls_apply_A(ft, uin)                # u_in + G (f u_in)
    iy = n // 2 - 1                                       # the plane y = 0
    cc = np.arange(n, dtype=np.float64) - n // 2 + 1
    Z, X = np.meshgrid(cc, cc, indexing="ij")
    pts = np.stack([X.ravel(), np.zeros(X.size), Z.ravel()], axis=1)
    ref = mie.total_field_points(k, eta_s / eta_b, radius, pts).reshape(n, n)
    ls = u[0, :, iy, :].cpu().numpy()
    bn = born[0, :, iy, :].cpu().numpy()
    e_ls = np.linalg.norm(ls - ref) / np.linalg.norm(ref)
    e_born = np.linalg.norm(bn - ref) / np.linalg.norm(ref)
    sc = ref - np.exp(1j * k * Z)                         # scattered part
    e_ls_sc = np.linalg.norm(ls - ref) / np.linalg.norm(sc)
    e_born_sc = np.linalg.norm(bn - ref) / np.linalg.norm(sc)
    print(f"[bead] n={n}, {info[0]['iters']} iterations: total-field error LS {e_ls:.3e}, Born {e_born:.3e}; "
          f"relative to the scattered field LS {e_ls_sc:.3e}, Born {e_born_sc:.3e}", flush=True)
    assert e_ls < 0.05 and e_ls < 0.2 * e_born
