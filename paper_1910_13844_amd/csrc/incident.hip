// Incident-field volumes from measured detector fields (Section "Computation of the 3D Incident
// Field"): angular-spectrum propagation of the field on the detector plane x3 = x_Gamma back to
// every slice z of the volume, with tilt transfer.
//
//   a      = y_in exp(-i x~.k~)                       (k_inc_demod; tilt transfer only)
//   A      = DFT2(a)                                   (FP64 2D DFTs of the kernel build)
//   B_z(w) = A(w) exp(-i (x_Gamma - z) sqrt(k^2 - |w + k~|^2)),  0 where |w + k~| > k   (k_inc_prop)
//   u_z    = IDFT2(B_z) exp(+i x~.k~)                  (k_inc_mod)
// The detector grid is the lateral voxel grid (spacing h = 1, positions i - n/2 + 1); the 2D
// convolution is periodic over it.  Without tilt transfer k~ = 0 in all three steps.  Everything
// runs in FP64 and is rounded once to the field precision.
#include <hip/hip_runtime.h>

#include "cplx.hpp"
#include "launch.hpp"

namespace ls {

static int inc_grid(size_t N) {
  const size_t b = (N + 255) / 256;
  return (int)(b < 16384 ? b : 16384);
}

template <typename T>
__global__ __launch_bounds__(256) void k_inc_demod(const cplx<T>* y, const double* kt, int tilt, cplx<double>* A,
                                                    int n, int Q) {
  const size_t M = (size_t)n * n;
  const size_t tot = M * Q;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < tot; i += (size_t)gridDim.x * 256) {
    const int q = (int)(i / M);
    const int iy = (int)((i / n) % n), ix = (int)(i % n);
    cplx<double> v = widen<double>(y[i]);
    if (tilt) {
      const double ph = -(kt[2 * q] * (ix - n / 2 + 1) + kt[2 * q + 1] * (iy - n / 2 + 1));
      double sn, cs;
      sincos(ph, &sn, &cs);
      v = v * cplx<double>{cs, sn};
    }
    A[i] = v;
  }
}

__global__ __launch_bounds__(256) void k_inc_prop(const cplx<double>* A, const double* kt, int tilt, double k,
                                                  double xg, cplx<double>* B, int n, int Q) {
  const size_t M = (size_t)n * n;
  const size_t tot = M * n * Q;
  const double two_pi_n = 2.0 * M_PI / n;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < tot; i += (size_t)gridDim.x * 256) {
    const int jx = (int)(i % n), jy = (int)((i / n) % n);
    const int iz = (int)((i / M) % n);
    const int q = (int)(i / (M * n));
    // DFT index -> angular frequency (index n/2 taken as -n/2)
    double wx = two_pi_n * (jx < n / 2 ? jx : jx - n);
    double wy = two_pi_n * (jy < n / 2 ? jy : jy - n);
    if (tilt) {
      wx += kt[2 * q];
      wy += kt[2 * q + 1];
    }
    const double s2 = k * k - (wx * wx + wy * wy);
    cplx<double> out = {0.0, 0.0};
    if (s2 >= 0.0) {
      const double dist = xg - (double)(iz - n / 2 + 1);
      double sn, cs;
      sincos(-dist * sqrt(s2), &sn, &cs);
      out = A[(size_t)q * M + (size_t)jy * n + jx] * cplx<double>{cs, sn};
    }
    B[i] = out;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_inc_mod(const cplx<double>* B, const double* kt, int tilt, cplx<T>* u, int n,
                                                  int Q) {
  const size_t M = (size_t)n * n;
  const size_t tot = M * n * Q;
  const double inv = 1.0 / (double)M;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < tot; i += (size_t)gridDim.x * 256) {
    const int ix = (int)(i % n), iy = (int)((i / n) % n);
    const int q = (int)(i / (M * n));
    cplx<double> v = inv * B[i];
    if (tilt) {
      const double ph = kt[2 * q] * (ix - n / 2 + 1) + kt[2 * q + 1] * (iy - n / 2 + 1);
      double sn, cs;
      sincos(ph, &sn, &cs);
      v = v * cplx<double>{cs, sn};
    }
    u[i] = narrow<T>(v);
  }
}

hipError_t launch_inc_demod(bool dbl, const void* y, const double* kt, int tilt, void* A, int n, int Q,
                            hipStream_t s) {
  const int g = inc_grid((size_t)n * n * Q);
  if (dbl)
    hipLaunchKernelGGL(k_inc_demod<double>, dim3(g), dim3(256), 0, s, (const cplx<double>*)y, kt, tilt,
                       (cplx<double>*)A, n, Q);
  else
    hipLaunchKernelGGL(k_inc_demod<float>, dim3(g), dim3(256), 0, s, (const cplx<float>*)y, kt, tilt,
                       (cplx<double>*)A, n, Q);
  return hipGetLastError();
}

hipError_t launch_inc_prop(const void* A, const double* kt, int tilt, double k, double xg, void* B, int n, int Q,
                           hipStream_t s) {
  const int g = inc_grid((size_t)n * n * n * Q);
  hipLaunchKernelGGL(k_inc_prop, dim3(g), dim3(256), 0, s, (const cplx<double>*)A, kt, tilt, k, xg, (cplx<double>*)B,
                     n, Q);
  return hipGetLastError();
}

hipError_t launch_inc_mod(bool dbl, const void* B, const double* kt, int tilt, void* u, int n, int Q, hipStream_t s) {
  const int g = inc_grid((size_t)n * n * n * Q);
  if (dbl)
    hipLaunchKernelGGL(k_inc_mod<double>, dim3(g), dim3(256), 0, s, (const cplx<double>*)B, kt, tilt,
                       (cplx<double>*)u, n, Q);
  else
    hipLaunchKernelGGL(k_inc_mod<float>, dim3(g), dim3(256), 0, s, (const cplx<double>*)B, kt, tilt, (cplx<float>*)u,
                       n, Q);
  return hipGetLastError();
}

}  // namespace ls
