"""Writes tests/golden/oracle_gm_fullsize.json: samples of the Proposition 2 kernel gm at the
full grid sizes with p = 4 (n = 144, 192, 256), from the oracle alone.

Calls only ``oracle`` and the shared input generators (n = 256 needs a few minutes and about
20 GB of host memory).  Run from the repository root:
    python tests/golden/make_gm_fullsize.py
For each n the file holds gm[d] at a fixed set of offsets d in [0, n-1]^3 (the corner cube of
Omega_{2n} reached by the response to a unit voxel at array index (0, 0, 0)): the origin, the
axes, the far corner and seeded random offsets.  The GPU's impulse response must reproduce them
(tests/test_gpu_big.py).
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import kernel  # noqa: E402
from paper_1910_13844_amd import workloads  # noqa: E402


def offsets(n):
    fixed = [(0, 0, 0), (0, 0, 1), (0, 1, 0), (1, 0, 0), (1, 1, 1), (0, 0, n - 1), (n - 1, 0, 0),
             (n // 2, n // 3, n // 5), (n - 1, n - 1, n - 1), (n - 2, 1, n - 1)]
    rng = np.random.default_rng(n)
    rnd = [tuple(int(t) for t in rng.integers(0, n, 3)) for _ in range(14)]
    return fixed + rnd


def main():
    k = workloads.k_of()
    out = {"k": k, "p": 4, "layout": "offsets (dz, dy, dx); gm[d] in the oracle's normalisation", "sizes": {}}
    for n in (144, 192, 256):
        gm = kernel.gm_coset(n, 4, k)
        offs = offsets(n)
        vals = [complex(gm[d]) for d in offs]
        out["sizes"][str(n)] = {"offsets": [list(d) for d in offs], "re": [v.real for v in vals],
                                "im": [v.imag for v in vals], "max_abs": float(np.max(np.abs(gm)))}
        print(n, vals[:3], flush=True)
        del gm
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_gm_fullsize.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
