// Detector-side operators of eq. (lipp2): far field on an m x m camera (m >= n pixels of the
// voxel spacing, both grids centred), the pupil / free-space propagation P, and decimation of the
// detector sampling.  FP64 pipelines on the 2D DFTs of the kernel build; inputs and outputs in the
// field precision.
//
// Far field, slice by slice (rectangle rule along z as in the square case):
//   Y = sum_z K^_z . DFT2(pad_M v_z),  y = crop_m IDFT2(Y),
// with K_z[t] = g(t - (m - n)/2, x_Gamma - z) on the M-periodic offset grid (M >= m + n - 1, so the
// circular convolution is the linear one on the kept pixels).  Its transpose correlates instead:
// K^_z evaluated at the negated frequency.  Pupil: pad to 2m, multiply by
// 1{|w| <= na k} exp(+-i dz sqrt(k^2 - |w|^2)) (conjugate for the adjoint), crop.
#include <hip/hip_runtime.h>

#include "cplx.hpp"
#include "launch.hpp"

namespace ls {

static int det_grid(size_t N) {
  const size_t b = (N + 255) / 256;
  return (int)(b < 16384 ? b : 16384);
}

// K[z][ty][tx] = exp(i k r) / (4 pi r), r = |(t - s) lateral, x_Gamma - z|
__global__ __launch_bounds__(256) void k_det_kernel(cplx<double>* K, int n, int M, int s, double k, double xg) {
  const size_t MM = (size_t)M * M;
  const size_t tot = MM * n;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < tot; i += (size_t)gridDim.x * 256) {
    const int tx = (int)(i % M), ty = (int)((i / M) % M), iz = (int)(i / MM);
    const int ox = (tx <= M - n ? tx : tx - M) - s;
    const int oy = (ty <= M - n ? ty : ty - M) - s;
    const double Z = xg - (double)(iz - n / 2 + 1);
    const double r = sqrt((double)ox * ox + (double)oy * oy + Z * Z);
    double sn, cs;
    sincos(k * r, &sn, &cs);
    const double a = 1.0 / (4.0 * M_PI * r);
    K[i] = {a * cs, a * sn};
  }
}

// V[z][j][i] = f . u at (j, i) < n, zero elsewhere
template <typename T>
__global__ __launch_bounds__(256) void k_det_pad_vol(const T* f, const cplx<T>* u, cplx<double>* V, int n, int M) {
  const size_t MM = (size_t)M * M;
  const size_t tot = MM * n;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < tot; i += (size_t)gridDim.x * 256) {
    const int x = (int)(i % M), y = (int)((i / M) % M), z = (int)(i / MM);
    cplx<double> v = {0.0, 0.0};
    if (x < n && y < n) {
      const size_t vi = ((size_t)z * n + y) * n + x;
      v = (double)f[vi] * widen<double>(u[vi]);
    }
    V[i] = v;
  }
}

// Q planes: P[q][j][i] = (conj?) y[q][j][i] for (j, i) < m, zero elsewhere
template <typename T>
__global__ __launch_bounds__(256) void k_det_pad2(const cplx<T>* y, cplx<double>* P, int m, int M, int Q, int cj) {
  const size_t MM = (size_t)M * M;
  const size_t tot = MM * Q;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < tot; i += (size_t)gridDim.x * 256) {
    const int x = (int)(i % M), yy = (int)((i / M) % M), q = (int)(i / MM);
    cplx<double> v = {0.0, 0.0};
    if (x < m && yy < m) {
      v = widen<double>(y[((size_t)q * m + yy) * m + x]);
      if (cj) v.im = -v.im;
    }
    P[i] = v;
  }
}

// Y[t] = sum_z K^_z[t] V^_z[t]
__global__ __launch_bounds__(256) void k_det_mulsum(const cplx<double>* K, const cplx<double>* V, cplx<double>* Y, int n,
                                                    int M) {
  const size_t MM = (size_t)M * M;
  for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < MM; t += (size_t)gridDim.x * 256) {
    cplx<double> acc = {0.0, 0.0};
    for (int z = 0; z < n; ++z) acc = acc + K[(size_t)z * MM + t] * V[(size_t)z * MM + t];
    Y[t] = acc;
  }
}

// V^_z[t] = K^_z[-t] R^[t]  (transpose: correlation)
__global__ __launch_bounds__(256) void k_det_mulT(const cplx<double>* K, const cplx<double>* R, cplx<double>* V, int n,
                                                  int M) {
  const size_t MM = (size_t)M * M;
  const size_t tot = MM * n;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < tot; i += (size_t)gridDim.x * 256) {
    const int tx = (int)(i % M), ty = (int)((i / M) % M), z = (int)(i / MM);
    const int nx = tx ? M - tx : 0, ny = ty ? M - ty : 0;
    V[i] = K[(size_t)z * MM + (size_t)ny * M + nx] * R[(size_t)ty * M + tx];
  }
}

// out[q][j][i] = scale * Y[q-plane][j][i] for (j, i) < m  (planes of size M^2, Q of them)
template <typename T>
__global__ __launch_bounds__(256) void k_det_crop(const cplx<double>* Y, cplx<T>* out, int m, int M, int Q,
                                                  double scale) {
  const size_t mm = (size_t)m * m;
  const size_t tot = mm * Q;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < tot; i += (size_t)gridDim.x * 256) {
    const int x = (int)(i % m), y = (int)((i / m) % m), q = (int)(i / mm);
    out[i] = narrow<T>(scale * Y[((size_t)q * M + y) * M + x]);
  }
}

// P[q][t] *= 1{|w| <= wc} exp(i sgn dz sqrt(k^2 - |w|^2))
__global__ __launch_bounds__(256) void k_det_pupil(cplx<double>* P, int M, int Q, double k, double wc, double dz,
                                                   int adjoint) {
  const size_t MM = (size_t)M * M;
  const size_t tot = MM * Q;
  const double two_pi_M = 2.0 * M_PI / M;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < tot; i += (size_t)gridDim.x * 256) {
    const int jx = (int)(i % M), jy = (int)((i / M) % M);
    const double wx = two_pi_M * (jx < M / 2 ? jx : jx - M);
    const double wy = two_pi_M * (jy < M / 2 ? jy : jy - M);
    const double r2 = wx * wx + wy * wy;
    cplx<double> v = {0.0, 0.0};
    if (r2 <= wc * wc) {
      const double kz = sqrt(fmax(k * k - r2, 0.0));
      double sn, cs;
      sincos(dz * kz, &sn, &cs);
      v = P[i] * cplx<double>{cs, adjoint ? -sn : sn};
    }
    P[i] = v;
  }
}

// decimation by q (keep pixels s + q i) and its transpose (zeros elsewhere)
template <typename T>
__global__ __launch_bounds__(256) void k_decimate(const cplx<T>* y, cplx<T>* out, int m, int q, int s, int Qn,
                                                  int transpose) {
  const int md = m / q;
  const size_t per = transpose ? (size_t)m * m : (size_t)md * md;
  const size_t tot = per * Qn;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < tot; i += (size_t)gridDim.x * 256) {
    const size_t pl = i / per;
    const size_t r = i % per;
    if (!transpose) {
      const int a = (int)(r % md), b = (int)(r / md);
      out[i] = y[pl * m * m + (size_t)(s + q * b) * m + (s + q * a)];
    } else {
      const int x = (int)(r % m), yy = (int)(r / m);
      const bool keep = x >= s && yy >= s && (x - s) % q == 0 && (yy - s) % q == 0 && (x - s) / q < md &&
                        (yy - s) / q < md;
      out[i] = keep ? y[pl * md * md + (size_t)((yy - s) / q) * md + (x - s) / q] : cplx<T>{T(0), T(0)};
    }
  }
}

hipError_t launch_det_kernel(void* K, int n, int M, int s, double k, double xg, hipStream_t st) {
  hipLaunchKernelGGL(k_det_kernel, dim3(det_grid((size_t)M * M * n)), dim3(256), 0, st, (cplx<double>*)K, n, M, s, k,
                     xg);
  return hipGetLastError();
}
hipError_t launch_det_pad_vol(bool dbl, const void* f, const void* u, void* V, int n, int M, hipStream_t st) {
  const int g = det_grid((size_t)M * M * n);
  if (dbl)
    hipLaunchKernelGGL(k_det_pad_vol<double>, dim3(g), dim3(256), 0, st, (const double*)f, (const cplx<double>*)u,
                       (cplx<double>*)V, n, M);
  else
    hipLaunchKernelGGL(k_det_pad_vol<float>, dim3(g), dim3(256), 0, st, (const float*)f, (const cplx<float>*)u,
                       (cplx<double>*)V, n, M);
  return hipGetLastError();
}
hipError_t launch_det_pad2(bool dbl, const void* y, void* P, int m, int M, int Q, int cj, hipStream_t st) {
  const int g = det_grid((size_t)M * M * Q);
  if (dbl)
    hipLaunchKernelGGL(k_det_pad2<double>, dim3(g), dim3(256), 0, st, (const cplx<double>*)y, (cplx<double>*)P, m, M,
                       Q, cj);
  else
    hipLaunchKernelGGL(k_det_pad2<float>, dim3(g), dim3(256), 0, st, (const cplx<float>*)y, (cplx<double>*)P, m, M, Q,
                       cj);
  return hipGetLastError();
}
hipError_t launch_det_mulsum(const void* K, const void* V, void* Y, int n, int M, hipStream_t st) {
  hipLaunchKernelGGL(k_det_mulsum, dim3(det_grid((size_t)M * M)), dim3(256), 0, st, (const cplx<double>*)K,
                     (const cplx<double>*)V, (cplx<double>*)Y, n, M);
  return hipGetLastError();
}
hipError_t launch_det_mulT(const void* K, const void* R, void* V, int n, int M, hipStream_t st) {
  hipLaunchKernelGGL(k_det_mulT, dim3(det_grid((size_t)M * M * n)), dim3(256), 0, st, (const cplx<double>*)K,
                     (const cplx<double>*)R, (cplx<double>*)V, n, M);
  return hipGetLastError();
}
hipError_t launch_det_crop(bool dbl, const void* Y, void* out, int m, int M, int Q, double scale, hipStream_t st) {
  const int g = det_grid((size_t)m * m * Q);
  if (dbl)
    hipLaunchKernelGGL(k_det_crop<double>, dim3(g), dim3(256), 0, st, (const cplx<double>*)Y, (cplx<double>*)out, m, M,
                       Q, scale);
  else
    hipLaunchKernelGGL(k_det_crop<float>, dim3(g), dim3(256), 0, st, (const cplx<double>*)Y, (cplx<float>*)out, m, M,
                       Q, scale);
  return hipGetLastError();
}
hipError_t launch_det_pupil(void* P, int M, int Q, double k, double wc, double dz, int adjoint, hipStream_t st) {
  hipLaunchKernelGGL(k_det_pupil, dim3(det_grid((size_t)M * M * Q)), dim3(256), 0, st, (cplx<double>*)P, M, Q, k, wc,
                     dz, adjoint);
  return hipGetLastError();
}
hipError_t launch_decimate(bool dbl, const void* y, void* out, int m, int q, int s, int Qn, int transpose,
                           hipStream_t st) {
  const size_t per = transpose ? (size_t)m * m : (size_t)(m / q) * (m / q);
  const int g = det_grid(per * Qn);
  if (dbl)
    hipLaunchKernelGGL(k_decimate<double>, dim3(g), dim3(256), 0, st, (const cplx<double>*)y, (cplx<double>*)out, m, q,
                       s, Qn, transpose);
  else
    hipLaunchKernelGGL(k_decimate<float>, dim3(g), dim3(256), 0, st, (const cplx<float>*)y, (cplx<float>*)out, m, q, s,
                       Qn, transpose);
  return hipGetLastError();
}

}  // namespace ls
