"""Writes tests/golden/oracle_bump_fullsize.json: the oracle's error of h^2 G v against the exact
continuous convolution of a radial bump (Theorem 1's accuracy statement) at n = 144, 192, 256 with
p = 4, at the three grid points the GPU test evaluates.

Calls only ``oracle`` (n = 256 needs several minutes and about 20 GB of host memory).  Run from the
repository root:
    python tests/golden/make_bump_fullsize.py
The error is not monotone in n (0.32e-9, 1.2e-11, 2.6e-11 at n = 96, 128, 144), so the GPU test
compares its errors with these instead of with a rate.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import bump, kernel, ops  # noqa: E402

L, KB, A, QEXP = 8.0, 1.3, 2.8, 4
PTS = [(0.0, 0.0, 0.0), (1.0, 1.0, -1.0), (2.0, -1.0, 1.0)]


def main():
    refs = [bump.conv_exact(float(np.sqrt(x * x + y * y + z * z)), KB, A, QEXP) for (x, y, z) in PTS]
    out = {"L": L, "kb": KB, "a": A, "q": QEXP, "p": 4, "points_zyx": [list(p[::-1]) for p in PTS], "err": {}}
    for n in (144, 192, 256):
        h = L / n
        gh = kernel.ghat_m(n, 4, KB * h)
        c = (np.arange(n) - n // 2 + 1) * h
        r = np.sqrt(c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2)
        Gv = h * h * ops.G_fft(gh, bump.bump(r, A, QEXP).astype(np.complex128))
        del gh, r
        errs = []
        for (x, y, z), ref in zip(PTS, refs):
            i = tuple(int(round(t / h)) + n // 2 - 1 for t in (z, y, x))
            errs.append(float(abs(Gv[i] - ref) / abs(ref)))
        out["err"][str(n)] = errs
        print(n, errs, flush=True)
        del Gv
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_bump_fullsize.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
