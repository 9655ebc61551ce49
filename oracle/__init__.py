"""CPU FP64 oracle for the Lippmann-Schwinger forward model (arXiv 1910.13844).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls or links this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the HIP library; the only module both
sides use is ``paper_1910_13844_amd.workloads`` (seeded input generators, none of the
method's arithmetic).

Everything is plain NumPy/SciPy in complex128/float64, in voxel units (h = 1):
k = k_b h, L = n, R = sqrt(3) n, delta = 2 pi / (n p), f~ = f h^2.

Modules
  dft       the DFT and its inverse (scipy.fft over the host cores)
  green     truncated Green function in Fourier, eqs. (GreenL), (GreenL2)
  kernel    Theorem 1 samples and the Proposition 2 modified kernel (two ways)
  ops       the discrete operator G: FFT form, Theorem 1 form, direct sum, dense matrix
  incident  plane-wave incident fields
  solver    BiCGSTAB for (I - G diag f) u = u_in, and a dense solve
  farfield  the detector operator G~ (brute-force sum and padded-FFT form) and its transpose
  grad      data term, its gradient (two forms) and finite differences
  mie       Mie series for a penetrable sphere (scalar wave)
  bump      closed-form continuous convolution of g with a radial bump (accuracy reference)

Every function that is pinned by an independent check says so in its docstring; the
checks live in tests/test_oracle_*.py.  Parity unpinned: none of the functions here
(the Mie comparison is a physics check whose tolerance the paper does not state; see
``mie``).
"""
