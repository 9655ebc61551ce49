"""Pins for oracle.mie (boundary conditions, trivial sphere) and the physics check of the
discrete LS solution against it (Fig. 2 of the paper, which prints no numbers: the check is
that the discrete solution approaches the analytical one as the grid is refined)."""
import numpy as np
import pytest
from scipy import special as sp

from oracle import incident, kernel, mie, ops, solver


def test_boundary_conditions_hold():
    k, k1, a = 1.0469375, 1.0469375 * 1.36 / 1.333, 10.0
    A, B = mie.coefficients(k, k1, a, mie.default_lmax(k, k1, a))
    for l in range(len(A)):
        h = sp.spherical_jn(l, k * a) + 1j * sp.spherical_yn(l, k * a)
        hp = sp.spherical_jn(l, k * a, True) + 1j * sp.spherical_yn(l, k * a, True)
        out = sp.spherical_jn(l, k * a) + A[l] * h
        inn = B[l] * sp.spherical_jn(l, k1 * a)
        dout = k * (sp.spherical_jn(l, k * a, True) + A[l] * hp)
        dinn = k1 * B[l] * sp.spherical_jn(l, k1 * a, True)
        assert abs(out - inn) <= 1e-12 * max(1, abs(out))
        assert abs(dout - dinn) <= 1e-12 * max(1, abs(dout))


def test_index_matched_sphere_is_transparent():
    k = 0.9
    pts = np.random.default_rng(0).uniform(-5, 5, (50, 3))
    u = mie.total_field_points(k, 1.0, 3.0, pts)
    assert np.max(np.abs(u - np.exp(1j * k * pts[:, 2]))) < 1e-12


@pytest.mark.slow
def test_ls_solution_approaches_mie_with_refinement():
    # physical sphere of radius 2.5 (in units of the coarse voxel), eta ratio 1.05, k = 1.0;
    # refine h by 2 and check that the relative L2 error inside the box decreases.
    kb, ratio, a, L = 1.0, 1.05, 2.5, 8.0
    errs = []
    for n in (8, 16):
        h = L / n
        c = (np.arange(n) - n // 2 + 1) * h
        Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
        inside = np.sqrt(X ** 2 + Y ** 2 + Z ** 2) <= a
        f = np.where(inside, (kb * h) ** 2 * (ratio ** 2 - 1.0), 0.0)
        gh = kernel.ghat_m(n, 4, kb * h)
        b = incident.plane_wave(n, kb * h, [0, 0, 1])
        u, info = solver.bicgstab(lambda v: ops.A_apply(gh, f, v), b, 1e-12)
        ref = mie.total_field_points(kb, ratio, a, np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)).reshape(u.shape)
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref - b))
    assert errs[1] < errs[0]
