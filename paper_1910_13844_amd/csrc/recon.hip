// Kernels of the reconstruction step (Algorithm 1, Section "Optimization"): the proximity
// operator of lam TV + i_{>=0} by fast gradient projection on its dual, the extrapolation of the
// accelerated iteration, and the TV value.
//
// TV is isotropic with forward differences (Dx)_v = (x_v - x_{v+e_z}, x_v - x_{v+e_y},
// x_v - x_{v+e_x}), a difference leaving the grid being 0.  Dual fields p, r hold three
// components [3][n^3]; components on the far faces stay 0.  One step of the method:
//   x_r   = P_C(b - lam D^T r)                       (k_prox_primal)
//   p_new = P_unit-ball(r + D x_r / (12 lam))         (k_prox_dual; 12 bounds ||D||^2 in 3D)
//   r     = p_new + beta (p_new - p_old),  p_old = p_new
// and the result is P_C(b - lam D^T p).  Memory-bound stencils: each thread owns one voxel,
// consecutive threads consecutive x, so all loads are coalesced; the +-1 neighbours along y and z
// are rows and planes that the same or adjacent workgroups just read (L2).
#include "cplx.hpp"
#include "launch.hpp"

namespace ls {

#define LS_GLOBAL __attribute__((address_space(1)))

template <typename T>
__global__ __launch_bounds__(256) void k_prox_init(const T* v, const T* d, T gamma, T* z, T* p, T* r, size_t N) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (size_t)gridDim.x * 256) {
    z[i] = d ? v[i] - gamma * d[i] : v[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      p[c * N + i] = T(0);
      r[c * N + i] = T(0);
    }
  }
}

// x = P_C(b - lam D^T q)
template <typename T>
__global__ __launch_bounds__(256) void k_prox_primal(const T* b, const T* q, T lam, int nonneg, T* x, int n) {
  const size_t N = (size_t)n * n * n;
  const size_t nn = (size_t)n * n;
  for (size_t v = (size_t)blockIdx.x * 256 + threadIdx.x; v < N; v += (size_t)gridDim.x * 256) {
    const int ix = (int)(v % n), iy = (int)((v / n) % n), iz = (int)(v / nn);
    const LS_GLOBAL T* q0 = (const LS_GLOBAL T*)q;
    const LS_GLOBAL T* q1 = q0 + N;
    const LS_GLOBAL T* q2 = q1 + N;
    // D^T q at v: q_c(v) where the difference from v exists, minus q_c(v - e_c) where that one does
    T dt = T(0);
    if (iz < n - 1) dt += q0[v];
    if (iy < n - 1) dt += q1[v];
    if (ix < n - 1) dt += q2[v];
    if (iz > 0) dt -= q0[v - nn];
    if (iy > 0) dt -= q1[v - n];
    if (ix > 0) dt -= q2[v - 1];
    T val = b[v] - lam * dt;
    if (nonneg && !(val > T(0))) val = T(0);
    x[v] = val;
  }
}

// p_new = P(r + step D x); r = p_new + beta (p_new - p); p = p_new
template <typename T>
__global__ __launch_bounds__(256) void k_prox_dual(const T* x, T* p, T* r, T step, T beta, int n) {
  const size_t N = (size_t)n * n * n;
  const size_t nn = (size_t)n * n;
  for (size_t v = (size_t)blockIdx.x * 256 + threadIdx.x; v < N; v += (size_t)gridDim.x * 256) {
    const int ix = (int)(v % n), iy = (int)((v / n) % n), iz = (int)(v / nn);
    const LS_GLOBAL T* xg = (const LS_GLOBAL T*)x;
    const T xv = xg[v];
    const T g0 = iz < n - 1 ? xv - xg[v + nn] : T(0);
    const T g1 = iy < n - 1 ? xv - xg[v + n] : T(0);
    const T g2 = ix < n - 1 ? xv - xg[v + 1] : T(0);
    T u0 = iz < n - 1 ? r[v] + step * g0 : T(0);
    T u1 = iy < n - 1 ? r[N + v] + step * g1 : T(0);
    T u2 = ix < n - 1 ? r[2 * N + v] + step * g2 : T(0);
    const T nrm = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
    if (nrm > T(1)) {
      const T s = T(1) / nrm;
      u0 *= s;
      u1 *= s;
      u2 *= s;
    }
    const T o0 = p[v], o1 = p[N + v], o2 = p[2 * N + v];
    p[v] = u0;
    p[N + v] = u1;
    p[2 * N + v] = u2;
    r[v] = u0 + beta * (u0 - o0);
    r[N + v] = u1 + beta * (u1 - o1);
    r[2 * N + v] = u2 + beta * (u2 - o2);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_extrapolate(const T* f, const T* fp, T beta, T* out, size_t N) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (size_t)gridDim.x * 256)
    out[i] = f[i] + beta * (f[i] - fp[i]);
}

// per-block FP64 partial sums of ||(Dx)_v||_2, then one block adds them in a fixed order
template <typename T>
__global__ __launch_bounds__(256) void k_tv_partial(const T* x, int n, double* part) {
  __shared__ double red[4];
  const size_t N = (size_t)n * n * n;
  const size_t nn = (size_t)n * n;
  double acc = 0.0;
  for (size_t v = (size_t)blockIdx.x * 256 + threadIdx.x; v < N; v += (size_t)gridDim.x * 256) {
    const int ix = (int)(v % n), iy = (int)((v / n) % n), iz = (int)(v / nn);
    const double xv = x[v];
    const double g0 = iz < n - 1 ? xv - (double)x[v + nn] : 0.0;
    const double g1 = iy < n - 1 ? xv - (double)x[v + n] : 0.0;
    const double g2 = ix < n - 1 ? xv - (double)x[v + 1] : 0.0;
    acc += sqrt(g0 * g0 + g1 * g1 + g2 * g2);
  }
  double vv[1] = {acc};
  block_sum<1>(vv, red);
  if (threadIdx.x == 0) part[blockIdx.x] = vv[0];
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* part, int nb, double* out) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) acc += part[i];
  double vv[1] = {acc};
  block_sum<1>(vv, red);
  if (threadIdx.x == 0) out[0] = vv[0];
}

static int grid_for(size_t N) {
  const size_t b = (N + 255) / 256;
  return (int)(b < 8192 ? b : 8192);
}

int tv_partial_blocks(size_t N) { return grid_for(N); }

hipError_t launch_prox_init(bool dbl, const void* v, const void* d, double gamma, void* z, void* p, void* r,
                            size_t N, hipStream_t s) {
  if (dbl)
    hipLaunchKernelGGL(k_prox_init<double>, dim3(grid_for(N)), dim3(256), 0, s, (const double*)v, (const double*)d,
                       gamma, (double*)z, (double*)p, (double*)r, N);
  else
    hipLaunchKernelGGL(k_prox_init<float>, dim3(grid_for(N)), dim3(256), 0, s, (const float*)v, (const float*)d,
                       (float)gamma, (float*)z, (float*)p, (float*)r, N);
  return hipGetLastError();
}

hipError_t launch_prox_primal(bool dbl, const void* b, const void* q, double lam, int nonneg, void* x, int n,
                              hipStream_t s) {
  const size_t N = (size_t)n * n * n;
  if (dbl)
    hipLaunchKernelGGL(k_prox_primal<double>, dim3(grid_for(N)), dim3(256), 0, s, (const double*)b, (const double*)q,
                       lam, nonneg, (double*)x, n);
  else
    hipLaunchKernelGGL(k_prox_primal<float>, dim3(grid_for(N)), dim3(256), 0, s, (const float*)b, (const float*)q,
                       (float)lam, nonneg, (float*)x, n);
  return hipGetLastError();
}

hipError_t launch_prox_dual(bool dbl, const void* x, void* p, void* r, double step, double beta, int n, hipStream_t s) {
  const size_t N = (size_t)n * n * n;
  if (dbl)
    hipLaunchKernelGGL(k_prox_dual<double>, dim3(grid_for(N)), dim3(256), 0, s, (const double*)x, (double*)p,
                       (double*)r, step, beta, n);
  else
    hipLaunchKernelGGL(k_prox_dual<float>, dim3(grid_for(N)), dim3(256), 0, s, (const float*)x, (float*)p, (float*)r,
                       (float)step, (float)beta, n);
  return hipGetLastError();
}

hipError_t launch_extrapolate(bool dbl, const void* f, const void* fp, double beta, void* out, size_t N,
                              hipStream_t s) {
  if (dbl)
    hipLaunchKernelGGL(k_extrapolate<double>, dim3(grid_for(N)), dim3(256), 0, s, (const double*)f,
                       (const double*)fp, beta, (double*)out, N);
  else
    hipLaunchKernelGGL(k_extrapolate<float>, dim3(grid_for(N)), dim3(256), 0, s, (const float*)f, (const float*)fp,
                       (float)beta, (float*)out, N);
  return hipGetLastError();
}

hipError_t launch_tv_value(bool dbl, const void* x, int n, double* part, double* out, hipStream_t s) {
  const size_t N = (size_t)n * n * n;
  const int nb = grid_for(N);
  if (dbl)
    hipLaunchKernelGGL(k_tv_partial<double>, dim3(nb), dim3(256), 0, s, (const double*)x, n, part);
  else
    hipLaunchKernelGGL(k_tv_partial<float>, dim3(nb), dim3(256), 0, s, (const float*)x, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, nb, out);
  return hipGetLastError();
}

}  // namespace ls
