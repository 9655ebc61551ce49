"""Discrete Fourier transforms used by the oracle: scipy.fft over all host cores.

Oracle module: test infrastructure only.

Unnormalised forward DFT with exp(-2 j pi k q / M) and an inverse carrying 1/M per axis, the
conventions of the paper's appendix on DFTs (the NumPy/SciPy convention).  A library routine
serves as this step; ``WORKERS`` (the logical CPUs this process may run on) is the thread count
the oracle's timings report.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as _sf

WORKERS = len(os.sched_getaffinity(0))


def fftn(a: np.ndarray) -> np.ndarray:
    return _sf.fftn(a, workers=WORKERS)


def ifftn(a: np.ndarray) -> np.ndarray:
    return _sf.ifftn(a, workers=WORKERS)


def fft2(a: np.ndarray) -> np.ndarray:
    return _sf.fft2(a, workers=WORKERS)


def ifft2(a: np.ndarray) -> np.ndarray:
    return _sf.ifft2(a, workers=WORKERS)
