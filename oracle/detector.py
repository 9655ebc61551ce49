"""Detector-side operators: a camera larger than a face of the volume (m >= n pixels), the pupil /
free-space propagation P, and decimation of the detector sampling (eq. (lipp2); Sections "Green's
Function Discretization for the Measurements" and "Free-Space Propagation and Pupil Function").

Oracle module: test infrastructure only.

Far field on an m x m detector (pixel spacing h, m >= n, both grids centred: pixel a at lateral
position a - m/2 + 1, voxel b at b - n/2 + 1), with the reading of oracle.farfield:
    y[a] = sum_z sum_b g(pos_m(a) - pos_n(b), x_Gamma - z) v[z, b].
``farfield_wide_direct`` writes the double sum out; ``farfield_wide_fft`` evaluates each slice's
2D linear convolution with FFTs of size M >= m + n - 1 (offsets pos_m(a) - pos_n(b) range over
m + n - 1 values); ``farfield_wide_T`` is the transpose (no conjugation), as in the gradient.

Pupil / propagation (reading; the paper gives P only as the convolution with a kernel combining
the microscope's point-spread function and a free-space propagation, applied by a padded FFT):
    P y = crop_m IDFT_{2m}( p ⊙ DFT_{2m}(pad_{2m} y) ),   p(w) = 1{|w| <= na k} exp(i dz sqrt(k^2 - |w|^2)),
an ideal circular pupil of radius na k (na = numerical aperture over the background index) and a
propagation over dz voxels along +x3.  P^H uses conj(p).

Decimation (detector pixel h' = q h, "downsample the result by q"): keep every q-th pixel, the
kept set containing the pixel at lateral position 0; its adjoint puts the samples back, zeros
elsewhere.
"""
from __future__ import annotations

import numpy as np

from . import dft, green


def positions(m: int) -> np.ndarray:
    return np.arange(m, dtype=np.float64) - m // 2 + 1


def farfield_wide_direct(v: np.ndarray, k: float, xg: float, m: int) -> np.ndarray:
    """Brute-force double sum, tiny grids only.  v [z, y, x] (n^3) -> y [m, m]."""
    n = v.shape[0]
    pn, pm, zc = positions(n), positions(m), positions(n)
    out = np.zeros((m, m), dtype=np.complex128)
    for iz in range(n):
        Z = xg - zc[iz]
        for ay in range(m):
            dy = pm[ay] - pn
            for ax in range(m):
                dx = pm[ax] - pn
                r = np.sqrt(dy[:, None] ** 2 + dx[None, :] ** 2 + Z * Z)
                out[ay, ax] += np.sum(green.g_free(r, k) * v[iz])
    return out


def fft_size(m: int, n: int) -> int:
    """Smallest even size >= m + n - 1 (the oracle uses it directly; any such size gives the same result)."""
    M = m + n - 1
    return M + (M % 2)


def wide_kernels(n: int, m: int, k: float, xg: float, M: int) -> np.ndarray:
    """K[z][ty][tx] = g(t - (m - n)/2, x_Gamma - z) for circular offsets t (t = i - j mod M)."""
    s = (m - n) // 2
    t = np.arange(M)
    t = np.where(t <= M - n, t, t - M)            # offsets i - j lie in [-(n - 1), m - 1]
    d = (t - s).astype(np.float64)
    zc = positions(n)
    out = np.empty((n, M, M), dtype=np.complex128)
    for iz in range(n):
        Z = xg - zc[iz]
        out[iz] = green.g_free(np.sqrt(d[:, None] ** 2 + d[None, :] ** 2 + Z * Z), k)
    return out


def farfield_wide_fft(v: np.ndarray, k: float, xg: float, m: int) -> np.ndarray:
    n = v.shape[0]
    M = fft_size(m, n)
    Kh = dft.fft2(wide_kernels(n, m, k, xg, M))
    vp = np.zeros((n, M, M), dtype=np.complex128)
    vp[:, :n, :n] = v
    y = dft.ifft2(np.sum(Kh * dft.fft2(vp), axis=0))
    return y[:m, :m]


def farfield_wide_T(r: np.ndarray, k: float, xg: float, n: int) -> np.ndarray:
    """(G~^T r)[z, b] = sum_a g(pos_m(a) - pos_n(b), x_Gamma - z) r[a]  (no conjugation)."""
    m = r.shape[0]
    M = fft_size(m, n)
    Kh = dft.fft2(wide_kernels(n, m, k, xg, M))
    rp = np.zeros((M, M), dtype=np.complex128)
    rp[:m, :m] = r
    # transpose of a circular convolution = circular correlation: kernel at negated frequencies
    Kneg = np.roll(Kh[:, ::-1, ::-1], 1, axis=(1, 2))
    out = dft.ifft2(Kneg * dft.fft2(rp)[None])
    return out[:, :n, :n]


def pupil_filter(M: int, k: float, na: float, dz: float) -> np.ndarray:
    w = 2.0 * np.pi * np.fft.fftfreq(M)
    r2 = w[:, None] ** 2 + w[None, :] ** 2
    inside = r2 <= (na * k) ** 2
    kz = np.sqrt(np.maximum(k * k - r2, 0.0))
    return np.where(inside, np.exp(1j * dz * kz), 0.0)


def pupil(y: np.ndarray, k: float, na: float, dz: float, adjoint: bool = False) -> np.ndarray:
    m = y.shape[-1]
    p = pupil_filter(2 * m, k, na, dz)
    if adjoint:
        p = np.conj(p)
    yp = np.zeros(y.shape[:-2] + (2 * m, 2 * m), dtype=np.complex128)
    yp[..., :m, :m] = y
    return dft.ifft2(p * dft.fft2(yp))[..., :m, :m]


def decimation_offset(m: int, q: int) -> int:
    """First kept index: the pixel at position 0 (index m/2 - 1) is kept."""
    return (m // 2 - 1) % q


def decimate(y: np.ndarray, q: int) -> np.ndarray:
    m = y.shape[-1]
    s = decimation_offset(m, q)
    return y[..., s::q, s::q]


def decimate_T(yd: np.ndarray, q: int, m: int) -> np.ndarray:
    s = decimation_offset(m, q)
    out = np.zeros(yd.shape[:-2] + (m, m), dtype=np.complex128)
    out[..., s::q, s::q] = yd
    return out


# ---------------------------------------------------------------------------------------------
# Forward model and Jacobian-adjoint product through a detector chain B = D_q P G~_m:
#   y_q = B (f . u_q),  u_q = (I - G diag f)^{-1} u_in,q,
#   Re(J^* gy) = sum_q Re(u_q . w_q),  (I - G diag f) w_q = G~_m^T conj(P^H D_q^T gy_q),
# the same conjugation argument as oracle.grad (G complex symmetric).  ``problem`` is an
# oracle.grad.Problem (solves with its kernel and tolerance).

def chain_forward(problem, f, dirs, m, na=None, dz=0.0, q=1):
    us, ys = [], []
    for d in dirs:
        u, _ = problem.total_field(f, d)
        y = farfield_wide_fft(f * u, problem.k, problem.xg, m)
        if na is not None:
            y = pupil(y, problem.k, na, dz)
        if q > 1:
            y = decimate(y, q)
        us.append(u)
        ys.append(y)
    return np.array(us), np.array(ys)


def chain_vjp(problem, f, us, gys, m, na=None, dz=0.0, q=1):
    from . import solver
    g = np.zeros(f.shape, dtype=np.float64)
    for u, gy in zip(us, gys):
        h = decimate_T(gy, q, m) if q > 1 else gy
        if na is not None:
            h = pupil(h, problem.k, na, dz, adjoint=True)
        b = farfield_wide_T(np.conj(h), problem.k, problem.xg, problem.n)
        w, _ = solver.bicgstab(problem.A(f), b, problem.tol, problem.maxit)
        g += np.real(u * w)
    return g
