// Complex arithmetic and wavefront helpers for the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ls {

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T re, im;
};

template <typename T>
__device__ __host__ __forceinline__ cplx<T> mk(T a, T b) { return cplx<T>{a, b}; }
template <typename T>
__device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cplx<T> operator*(T s, cplx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> conj(cplx<T> a) { return {a.re, -a.im}; }
// a * conj(b)
template <typename T>
__device__ __forceinline__ cplx<T> mulc(cplx<T> a, cplx<T> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// multiply by +i (DIR=+1) or -i (DIR=-1)
template <int DIR, typename T>
__device__ __forceinline__ cplx<T> mul_i(cplx<T> a) {
  return DIR > 0 ? cplx<T>{-a.im, a.re} : cplx<T>{a.im, -a.re};
}
template <typename T>
__device__ __forceinline__ T norm2(cplx<T> a) { return a.re * a.re + a.im * a.im; }

template <typename D, typename T>
__device__ __forceinline__ cplx<D> widen(cplx<T> a) { return {(D)a.re, (D)a.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> narrow(cplx<double> a) { return {(T)a.re, (T)a.im}; }

// conj(a) * b accumulated in FP64 (inner product <a, b> = sum conj(a) b)
template <typename T>
__device__ __forceinline__ void dot_acc(cplx<double>& acc, cplx<T> a, cplx<T> b) {
  double ar = a.re, ai = a.im, br = b.re, bi = b.im;
  acc.re += ar * br + ai * bi;
  acc.im += ar * bi - ai * br;
}

// Orders the LDS traffic of a wavefront around this point for lanes that exchange data through
// LDS.  The LDS unit executes the DS instructions of one wavefront in issue order, so it is
// enough that the compiler keeps their program order here: a compiler barrier plus the
// wave-level scheduling barrier, without a hardware wait on outstanding LDS operations.
__device__ __forceinline__ void wave_sync() {
#ifdef LS_WAVE_FENCE
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#else
  asm volatile("" ::: "memory");
  __builtin_amdgcn_wave_barrier();
#endif
}

__device__ __forceinline__ double shfl_down_d(double v, int off) {
  return __shfl_down(v, off, 64);
}

// Block-wide deterministic sum of NV doubles per thread (fixed reduction order).
// `red` must hold NV * (blockDim/64) doubles.  Result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double x = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += shfl_down_d(x, off);
    v[k] = x;
  }
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[wid * NV + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[w * NV + k];
      v[k] = s;
    }
  }
}

}  // namespace ls
