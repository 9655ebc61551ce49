// In-LDS Stockham FFTs executed by a group of lanes inside one wavefront.
//
// A transform of length N is carried out by L = N/E lanes that each hold E elements in
// registers for the duration of a radix pass: every pass loads all N values, applies the
// twiddles and radix-R butterflies, and stores them back in place.  Because the L lanes sit in
// one wavefront (L divides 64) and LDS requests of a wavefront execute in order, passes need no
// workgroup barrier, only a wavefront-level fence.
//
// Transforms are unnormalised: DIR = -1 computes X[k] = sum_j x[j] exp(-2 pi i j k / N),
// DIR = +1 the same with exp(+...).  Twiddles come from a table tw[m] = exp(-2 pi i m / NT)
// (NT = N * TWS) held in LDS.
#pragma once
#include "cplx.hpp"

namespace ls {

// ---------------------------------------------------------------------------------------------
// small DFTs on registers
template <int R, int DIR, typename T>
struct SmallDFT;

template <int DIR, typename T>
struct SmallDFT<2, DIR, T> {
  static __device__ __forceinline__ void run(cplx<T>* a) {
    cplx<T> t = a[0] - a[1];
    a[0] = a[0] + a[1];
    a[1] = t;
  }
};

template <int DIR, typename T>
struct SmallDFT<3, DIR, T> {
  static __device__ __forceinline__ void run(cplx<T>* a) {
    const T c = (T)-0.5;
    const T s = (T)(DIR * 0.86602540378443864676);
    cplx<T> t1 = a[1] + a[2];
    cplx<T> t2 = a[1] - a[2];
    cplx<T> m = a[0] + c * t1;
    cplx<T> is2 = {-s * t2.im, s * t2.re};  // i * s * t2
    a[0] = a[0] + t1;
    a[1] = m + is2;
    a[2] = m - is2;
  }
};

template <int DIR, typename T>
struct SmallDFT<4, DIR, T> {
  static __device__ __forceinline__ void run(cplx<T>* a) {
    cplx<T> s02 = a[0] + a[2], d02 = a[0] - a[2];
    cplx<T> s13 = a[1] + a[3], d13 = mul_i<DIR>(a[1] - a[3]);
    a[0] = s02 + s13;
    a[2] = s02 - s13;
    a[1] = d02 + d13;
    a[3] = d02 - d13;
  }
};

template <int DIR, typename T>
struct SmallDFT<8, DIR, T> {
  static __device__ __forceinline__ void run(cplx<T>* a) {
    cplx<T> e[4] = {a[0], a[2], a[4], a[6]};
    cplx<T> o[4] = {a[1], a[3], a[5], a[7]};
    SmallDFT<4, DIR, T>::run(e);
    SmallDFT<4, DIR, T>::run(o);
    const T h = (T)0.70710678118654752440;
    // w^k = exp(DIR i pi k / 4)
    cplx<T> o1 = {h * (o[1].re - DIR * o[1].im), h * (o[1].im + DIR * o[1].re)};
    cplx<T> o2 = mul_i<DIR>(o[2]);
    cplx<T> o3 = {h * (-o[3].re - DIR * o[3].im), h * (-o[3].im + DIR * o[3].re)};
    a[0] = e[0] + o[0];
    a[4] = e[0] - o[0];
    a[1] = e[1] + o1;
    a[5] = e[1] - o1;
    a[2] = e[2] + o2;
    a[6] = e[2] - o2;
    a[3] = e[3] + o3;
    a[7] = e[3] - o3;
  }
};

// ---------------------------------------------------------------------------------------------
// radix plans: (E, radices...).  Every radix divides E and N/E divides 64.
template <int N>
struct Plan;
template <> struct Plan<8>   { static constexpr int E = 8;  static constexpr int NP = 1; static constexpr int R[5] = {8, 1, 1, 1, 1}; };
template <> struct Plan<16>  { static constexpr int E = 8;  static constexpr int NP = 2; static constexpr int R[5] = {8, 2, 1, 1, 1}; };
template <> struct Plan<32>  { static constexpr int E = 8;  static constexpr int NP = 2; static constexpr int R[5] = {8, 4, 1, 1, 1}; };
template <> struct Plan<64>  { static constexpr int E = 8;  static constexpr int NP = 2; static constexpr int R[5] = {8, 8, 1, 1, 1}; };
template <> struct Plan<128> { static constexpr int E = 8;  static constexpr int NP = 3; static constexpr int R[5] = {8, 8, 2, 1, 1}; };
template <> struct Plan<256> { static constexpr int E = 8;  static constexpr int NP = 3; static constexpr int R[5] = {8, 8, 4, 1, 1}; };
template <> struct Plan<512> { static constexpr int E = 8;  static constexpr int NP = 3; static constexpr int R[5] = {8, 8, 8, 1, 1}; };
template <> struct Plan<96>  { static constexpr int E = 12; static constexpr int NP = 4; static constexpr int R[5] = {3, 4, 4, 2, 1}; };
template <> struct Plan<192> { static constexpr int E = 12; static constexpr int NP = 4; static constexpr int R[5] = {3, 4, 4, 4, 1}; };
template <> struct Plan<384> { static constexpr int E = 12; static constexpr int NP = 5; static constexpr int R[5] = {3, 4, 4, 4, 2}; };

template <int N>
struct Lanes {
  static constexpr int value = N / Plan<N>::E;
  static_assert(64 % (N / Plan<N>::E) == 0, "a transform must stay inside one wavefront");
};

// One Stockham pass: radix R after sub-transforms of size NS are complete.
template <typename T, int N, int E, int R, int NS, int DIR, int TWS>
__device__ __forceinline__ void stockham_pass(cplx<T>* base, int stride, int lane, const cplx<T>* tw) {
  constexpr int L = N / E;
  constexpr int NB = E / R;
  static_assert(E % R == 0, "radix must divide E");
  cplx<T> v[E];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lane + b * L;
#pragma unroll
    for (int r = 0; r < R; ++r) v[b * R + r] = base[(j + r * (N / R)) * stride];
  }
  wave_sync();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lane + b * L;
    const int k = j % NS;
    if (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const int m = r * k * (N / (NS * R));
        cplx<T> w = tw[m * TWS];
        if (DIR > 0) w.im = -w.im;
        v[b * R + r] = v[b * R + r] * w;
      }
    }
    SmallDFT<R, DIR, T>::run(&v[b * R]);
    const int o = (j / NS) * NS * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) base[(o + r * NS) * stride] = v[b * R + r];
  }
  wave_sync();
}

// Full transform of length N at base[i*stride] by lane `lane` in [0, N/E).
template <typename T, int N, int DIR, int TWS>
__device__ __forceinline__ void fft_group(cplx<T>* base, int stride, int lane, const cplx<T>* tw) {
  using P = Plan<N>;
  constexpr int E = P::E;
  wave_sync();
  stockham_pass<T, N, E, P::R[0], 1, DIR, TWS>(base, stride, lane, tw);
  if constexpr (P::NP > 1) stockham_pass<T, N, E, P::R[1], P::R[0], DIR, TWS>(base, stride, lane, tw);
  if constexpr (P::NP > 2) stockham_pass<T, N, E, P::R[2], P::R[0] * P::R[1], DIR, TWS>(base, stride, lane, tw);
  if constexpr (P::NP > 3)
    stockham_pass<T, N, E, P::R[3], P::R[0] * P::R[1] * P::R[2], DIR, TWS>(base, stride, lane, tw);
  if constexpr (P::NP > 4)
    stockham_pass<T, N, E, P::R[4], P::R[0] * P::R[1] * P::R[2] * P::R[3], DIR, TWS>(base, stride, lane, tw);
}

}  // namespace ls
