"""Writes tests/golden/oracle_values.json: regression values of the oracle.

Calls only ``oracle`` and the shared input generators.  Run from the repository root:
    python tests/golden/make_golden.py
The paper itself prints no numbers for the forward operator (its experiments are figures and
reconstruction errors), so these values are the oracle's own, frozen after its independent pins
(tests/test_oracle_*.py) passed; tests/test_golden.py checks the oracle still reproduces them.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import green, kernel, mie, ops  # noqa: E402
from paper_1910_13844_amd import workloads  # noqa: E402


def c(z):
    return [float(np.real(z)), float(np.imag(z))]


def main():
    out = {}
    k = workloads.k_of()
    # Fig. 2 geometry of the paper (bead in water): lambda = 532 nm, eta_b = 1.3388, h = lambda/16
    out["fig2_k_voxel"] = 2 * np.pi * 1.3388 / 16
    R8 = np.sqrt(3.0) * 8
    s = [0.0, 0.25, 0.5, k, 1.7, 3.0]
    out["ghat_t_n8"] = {"k": k, "R": R8, "s": s, "values": [c(v) for v in green.ghat_t(np.array(s), k, R8)]}
    gm = kernel.gm_coset(8, 4, k)
    pts = [(0, 0, 0), (1, 0, 0), (3, 2, 1), (8, 8, 8), (15, 1, 7)]
    out["gm_n8_p4"] = {"points": pts, "values": [c(gm[p]) for p in pts]}
    v = workloads.random_field(11, (8, 8, 8))
    Gv = ops.G_fft(np.fft.fftn(gm), v)
    out["Gv_n8_p4_seed11"] = {"points": pts[:3] + [(7, 7, 7)], "values": [c(Gv[p]) for p in pts[:3] + [(7, 7, 7)]]}
    k1 = k * 1.36 / 1.333
    A, B = mie.coefficients(k, k1, 10.0, 6)
    out["mie_sphere32"] = {"k": k, "k1": k1, "a": 10.0, "A": [c(a) for a in A], "B": [c(b) for b in B]}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_values.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
