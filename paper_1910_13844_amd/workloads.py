"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module generates *inputs* only: scattering potentials (phantoms), illumination
directions and the dimensionless geometry of a problem. It contains none of the
method's arithmetic (no Green function, no convolution, no solver, no incident field).

Units (Section "Continuous-Domain Formulation" and Theorem 1 of the paper): everything
is expressed in voxel units, h = 1.  With k_b = 2*pi*eta_b/lambda0 the dimensionless
wavenumber is k = k_b*h, and the dimensionless scattering potential is
f~ = f*h^2 = (2*pi*h/lambda0)^2 * (eta^2 - eta_b^2), since f = k_b^2 (eta^2/eta_b^2 - 1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Dict, Tuple

import numpy as np

ETA_B = 1.333          # background index used by every synthetic workload
H_OVER_LAMBDA = 1.0 / 8.0   # voxel = lambda0 / 8


def k_of(h_over_lambda: float = H_OVER_LAMBDA, eta_b: float = ETA_B) -> float:
    """Dimensionless background wavenumber k = k_b*h = 2*pi*eta_b*h/lambda0."""
    return 2.0 * math.pi * eta_b * h_over_lambda


def potential_from_index(eta: np.ndarray, h_over_lambda: float = H_OVER_LAMBDA,
                         eta_b: float = ETA_B) -> np.ndarray:
    """f~ = (2*pi*h/lambda0)^2 (eta^2 - eta_b^2): the input convention for the contrast."""
    c = (2.0 * math.pi * h_over_lambda) ** 2
    return c * (eta.astype(np.float64) ** 2 - eta_b ** 2)


def voxel_coords(n: int) -> np.ndarray:
    """Signed voxel positions i - n/2 + 1 for array index i in [0, n)."""
    return np.arange(n, dtype=np.float64) - n / 2 + 1


def sphere_index(n: int, radius: float, eta_s: float, eta_b: float = ETA_B) -> np.ndarray:
    """Binary voxelised sphere centred at x = 0 (array index n/2 - 1), |x| <= radius."""
    c = voxel_coords(n)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    inside = (x * x + y * y + z * z) <= radius * radius
    eta = np.full((n, n, n), eta_b, dtype=np.float64)
    eta[inside] = eta_s
    return eta


def sphere_potential(n: int, radius: float, eta_s: float, eta_b: float = ETA_B,
                     h_over_lambda: float = H_OVER_LAMBDA) -> np.ndarray:
    return potential_from_index(sphere_index(n, radius, eta_s, eta_b), h_over_lambda, eta_b)


def blob_index(seed: int, n: int, nblobs: int = 20, sigma_range: Tuple[float, float] = (3.0, 12.0),
               dn_max: float = 0.05, eta_b: float = ETA_B) -> np.ndarray:
    """Sum of Gaussian blobs over the background index.

    Draw order is fixed: centres ~ U[-n/4, n/4]^3 (voxel units, around x = 0), then
    sigma ~ U[sigma_range], then amplitudes ~ U[0, dn_max].  Not clipped.
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-n / 4, n / 4, size=(nblobs, 3))
    sigmas = rng.uniform(sigma_range[0], sigma_range[1], size=nblobs)
    amps = rng.uniform(0.0, dn_max, size=nblobs)
    c = voxel_coords(n)
    dn = np.zeros((n, n, n), dtype=np.float64)
    for (cz, cy, cx), s, a in zip(centres, sigmas, amps):
        gz = np.exp(-((c - cz) ** 2) / (2 * s * s))
        gy = np.exp(-((c - cy) ** 2) / (2 * s * s))
        gx = np.exp(-((c - cx) ** 2) / (2 * s * s))
        dn += a * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    return eta_b + dn


def blob_potential(seed: int, n: int, nblobs: int = 20, sigma_range=(3.0, 12.0), dn_max: float = 0.05,
                   eta_b: float = ETA_B, h_over_lambda: float = H_OVER_LAMBDA) -> np.ndarray:
    return potential_from_index(blob_index(seed, n, nblobs, sigma_range, dn_max, eta_b),
                                h_over_lambda, eta_b)


def cone_dirs(Q: int, theta_deg: float) -> np.ndarray:
    """Unit propagation directions on a cone of half-angle theta around +z, uniform azimuths."""
    th = math.radians(theta_deg)
    phi = 2.0 * math.pi * np.arange(Q) / Q
    return np.stack([math.sin(th) * np.cos(phi), math.sin(th) * np.sin(phi),
                     np.full(Q, math.cos(th))], axis=1)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int
    p: int
    Q: int
    theta_deg: float
    tol: float
    precision: str          # "c64" or "c128"
    phantom: str            # "sphere" or "blobs"
    seed: int = 0
    dn_max: float = 0.05
    kind: str = "forward"   # "forward": solves + far fields; "gradient": data-term gradient at f0

    @property
    def k(self) -> float:
        return k_of()

    @property
    def xg(self) -> float:
        """Detector plane position in voxel units (x_Gamma = L = n h)."""
        return float(self.n)

    def potential(self) -> np.ndarray:
        if self.phantom == "sphere":
            return sphere_potential(self.n, 10.0, 1.36)
        return blob_potential(self.seed, self.n, dn_max=self.dn_max)

    def dirs(self) -> np.ndarray:
        if self.Q == 1 and self.theta_deg == 0.0:
            return np.array([[0.0, 0.0, 1.0]])
        return cone_dirs(self.Q, self.theta_deg)


WORKLOADS: Dict[str, Workload] = {
    # 32^3 sphere (radius 10 voxels, eta 1.36), one plane wave along +z, complex128, tol 1e-8.
    "A": Workload("sphere32_c128", 32, 4, 1, 0.0, 1e-8, "c128", "sphere"),
    # 128^3 blob phantom, 60 illuminations on a 45 degree cone, complex64, tol 1e-5.
    "B": Workload("blobs128_q60_c64", 128, 4, 60, 45.0, 1e-5, "c64", "blobs", seed=0, dn_max=0.05),
    # 256^3 blob phantom with stronger contrast, 60 illuminations, complex64, tol 1e-5.
    "C": Workload("blobs256_q60_c64", 256, 4, 60, 45.0, 1e-5, "c64", "blobs", seed=1, dn_max=0.1),
    # 128^3 gradient workload, 40 illuminations on a 40 degree cone.
    # f0 = phantom seed 2; data from f0 + a 5-blob perturbation (seed 3) with 30 dB noise (seed 4).
    # Solver tolerance 1e-6: the gradient sums 40 views whose terms largely cancel, so at 1e-5 the
    # solves alone leave it ~7e-4 from the exact one; 1e-6 brings it within 1e-4.
    "D": Workload("grad128_q40_c64", 128, 4, 40, 40.0, 1e-6, "c64", "blobs", seed=2, dn_max=0.05,
                  kind="gradient"),
}


def perturbed_potential(n: int, seed_base: int = 2, seed_pert: int = 3) -> Tuple[np.ndarray, np.ndarray]:
    """f0 and f_true = f0 + small blob perturbation (5 blobs, sigma in [2, 5], dn_max 0.01)."""
    f0 = blob_potential(seed_base, n, dn_max=0.05)
    pert = blob_potential(seed_pert, n, nblobs=5, sigma_range=(2.0, 5.0), dn_max=0.01)
    return f0, f0 + pert


def add_noise(y: np.ndarray, seed: int = 4, snr_db: float = 30.0) -> np.ndarray:
    """Complex Gaussian noise per view at the given SNR: variance ||y_q||^2 / (M 10^(snr/10))."""
    rng = np.random.default_rng(seed)
    y = np.asarray(y)
    out = np.empty_like(y)
    for q in range(y.shape[0]):
        M = y[q].size
        var = float(np.vdot(y[q], y[q]).real) / (M * 10 ** (snr_db / 10.0))
        sd = math.sqrt(var / 2.0)
        out[q] = y[q] + sd * (rng.standard_normal(y[q].shape) + 1j * rng.standard_normal(y[q].shape))
    return out


def random_field(seed: int, shape, complex_: bool = True) -> np.ndarray:
    """Seeded standard-normal test vector (complex when requested)."""
    rng = np.random.default_rng(seed)
    if complex_:
        return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return rng.standard_normal(shape)


def view_subsets(Q: int, size: int, iters: int, seed: int) -> List[List[int]]:
    """Seeded view subsets for stochastic reconstruction: `size` distinct views per iteration, sorted."""
    rng = np.random.default_rng(seed)
    return [sorted(rng.choice(Q, size=size, replace=False).tolist()) for _ in range(iters)]
