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
template <> struct Plan<144> { static constexpr int E = 36; static constexpr int NP = 4; static constexpr int R[5] = {4, 4, 3, 3, 1}; };
template <> struct Plan<288> { static constexpr int E = 36; static constexpr int NP = 5; static constexpr int R[5] = {4, 4, 2, 3, 3}; };
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

// ---------------------------------------------------------------------------------------------
// 9-point DFT in registers as 3 x 3 (Cooley-Tukey): 3-point DFTs over n1 of x[3 n1 + n2], twiddles
// exp(DIR 2 pi i n2 k1 / 9), 3-point DFTs over n2; X[k1 + 3 k2].
template <int DIR, typename T>
struct SmallDFT<9, DIR, T> {
  static __device__ __forceinline__ void run(cplx<T>* a) {
    const T c1 = (T)0.76604444311897803520, s1 = (T)0.64278760968653932632;  // 2 pi / 9
    const T c2 = (T)0.17364817766693034885, s2 = (T)0.98480775301220805936;  // 4 pi / 9
    const T c4 = (T)-0.93969262078590838405, s4 = (T)0.34202014332566873304; // 8 pi / 9
    cplx<T> b[3][3];
#pragma unroll
    for (int n2 = 0; n2 < 3; ++n2) {
      cplx<T> t[3] = {a[n2], a[3 + n2], a[6 + n2]};
      SmallDFT<3, DIR, T>::run(t);
      b[n2][0] = t[0];
      b[n2][1] = t[1];
      b[n2][2] = t[2];
    }
    b[1][1] = b[1][1] * cplx<T>{c1, DIR * s1};
    b[1][2] = b[1][2] * cplx<T>{c2, DIR * s2};
    b[2][1] = b[2][1] * cplx<T>{c2, DIR * s2};
    b[2][2] = b[2][2] * cplx<T>{c4, DIR * s4};
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      cplx<T> t[3] = {b[0][k1], b[1][k1], b[2][k1]};
      SmallDFT<3, DIR, T>::run(t);
      a[k1] = t[0];
      a[k1 + 3] = t[1];
      a[k1 + 6] = t[2];
    }
  }
};

// 12-point DFT by the prime-factor algorithm, 12 = 3 x 4: input n = (4 n1 + 3 n2) mod 12, 4-point
// DFTs over n2, 3-point DFTs over n1, output k = (4 k1 + 9 k2) mod 12.
template <int DIR, typename T>
struct SmallDFT<12, DIR, T> {
  static __device__ __forceinline__ void run(cplx<T>* a) {
    cplx<T> y[3][4];
#pragma unroll
    for (int n1 = 0; n1 < 3; ++n1) {
#pragma unroll
      for (int n2 = 0; n2 < 4; ++n2) y[n1][n2] = a[(4 * n1 + 3 * n2) % 12];
      SmallDFT<4, DIR, T>::run(y[n1]);
    }
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
      cplx<T> t[3] = {y[0][k2], y[1][k2], y[2][k2]};
      SmallDFT<3, DIR, T>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < 3; ++k1) a[(4 * k1 + 9 * k2) % 12] = t[k1];
    }
  }
};

// 36-point DFT by the prime-factor algorithm, 36 = 4 x 9: input n = (9 n1 + 4 n2) mod 36, 9-point
// DFTs over n2, 4-point DFTs over n1, output k = (9 k1 + 28 k2) mod 36.
template <int DIR, typename T>
struct SmallDFT<36, DIR, T> {
  static __device__ __forceinline__ void run(cplx<T>* a) {
    cplx<T> y[4][9];
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) {
#pragma unroll
      for (int n2 = 0; n2 < 9; ++n2) y[n1][n2] = a[(9 * n1 + 4 * n2) % 36];
      SmallDFT<9, DIR, T>::run(y[n1]);
    }
#pragma unroll
    for (int k2 = 0; k2 < 9; ++k2) {
      cplx<T> t[4] = {y[0][k2], y[1][k2], y[2][k2], y[3][k2]};
      SmallDFT<4, DIR, T>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) a[(9 * k1 + 28 * k2) % 36] = t[k1];
    }
  }
};

// ---------------------------------------------------------------------------------------------
// 24-point DFT in registers by the prime-factor (Good-Thomas) algorithm, 24 = 3 x 8 with 3 and 8
// coprime, so no twiddles: input n = (8 n1 + 3 n2) mod 24, 8-point DFTs over n2, 3-point DFTs over
// n1, output k = (16 k1 + 9 k2) mod 24 (k = k1 mod 3, k = k2 mod 8).  Index maps are
// compile-time, so the permutations cost nothing.
template <int DIR, typename T>
struct SmallDFT<24, DIR, T> {
  static __device__ __forceinline__ void run(cplx<T>* a) {
    cplx<T> y[3][8];
#pragma unroll
    for (int n1 = 0; n1 < 3; ++n1) {
#pragma unroll
      for (int n2 = 0; n2 < 8; ++n2) y[n1][n2] = a[(8 * n1 + 3 * n2) % 24];
      SmallDFT<8, DIR, T>::run(y[n1]);
    }
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
      cplx<T> t[3] = {y[0][k2], y[1][k2], y[2][k2]};
      SmallDFT<3, DIR, T>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < 3; ++k1) a[(16 * k1 + 9 * k2) % 24] = t[k1];
    }
  }
};

// ---------------------------------------------------------------------------------------------
// 16-point DFT in registers as 4 x 4 with internal twiddles exp(DIR 2 pi i m / 16).
template <int DIR, typename T>
struct SmallDFT<16, DIR, T> {
  static __device__ __forceinline__ void run(cplx<T>* a) {
    const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173, h = (T)0.70710678118654752440;
    // w16^m for m = 0..9
    const cplx<T> w[10] = {{(T)1, (T)0},       {c1, DIR * s1},  {h, DIR * h},     {s1, DIR * c1},   {(T)0, (T)DIR},
                           {-s1, DIR * c1},    {-h, DIR * h},   {-c1, DIR * s1},  {(T)-1, (T)0},    {-c1, -DIR * s1}};
    cplx<T> b[16];
#pragma unroll
    for (int j1 = 0; j1 < 4; ++j1) {
      cplx<T> t[4] = {a[j1], a[j1 + 4], a[j1 + 8], a[j1 + 12]};
      SmallDFT<4, DIR, T>::run(t);
      b[j1 * 4 + 0] = t[0];
#pragma unroll
      for (int k = 1; k < 4; ++k) b[j1 * 4 + k] = j1 == 0 ? t[k] : t[k] * w[j1 * k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      cplx<T> t[4] = {b[k], b[4 + k], b[8 + k], b[12 + k]};
      SmallDFT<4, DIR, T>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) a[k + 4 * k2] = t[k2];
    }
  }
};

template <int DIR, typename T>
struct SmallDFT<1, DIR, T> {
  static __device__ __forceinline__ void run(cplx<T>*) {}
};

// ---------------------------------------------------------------------------------------------
// Register-resident transforms with a single LDS transpose (four-step, N = L * E).
// Layout A: lane l in [0, L) holds a[j] = x[l + L j], j < E (natural index l + L j).
// Layout B: lane l holds a[t L + k2] = X[k1 + E k2] for k1 = l P + t (t < P = E / L), k2 < L.
// fft_a2b maps layout A data to its transform in layout B; fft_b2a is the inverse structure
// (layout B spectrum -> layout A signal).  Both are unnormalised, with sign DIR.  The L lanes
// of a transform must sit in one wavefront; `buf` (N entries at stride s) is scratch for the
// transpose and may alias the data's own LDS storage.
template <int N>
struct Split;
template <> struct Split<8>   { static constexpr int L = 1, E = 8; };
template <> struct Split<16>  { static constexpr int L = 2, E = 8; };
template <> struct Split<32>  { static constexpr int L = 4, E = 8; };
template <> struct Split<64>  { static constexpr int L = 8, E = 8; };
template <> struct Split<128> { static constexpr int L = 8, E = 16; };
template <> struct Split<256> { static constexpr int L = 16, E = 16; };
template <> struct Split<96>  { static constexpr int L = 4, E = 24; };
template <> struct Split<192> { static constexpr int L = 8, E = 24; };
template <> struct Split<48>  { static constexpr int L = 4, E = 12; };
template <> struct Split<144> { static constexpr int L = 4, E = 36; };

template <int N>
__device__ __forceinline__ int tpos(int k1, int m) {
  // position of T[k1][m] in the scratch: row k1, column m swizzled by the reading lane
  constexpr int L = Split<N>::L, P = Split<N>::E / Split<N>::L;
  return k1 * L + (m ^ ((k1 / P) & (L - 1)));
}

// Storage order of a layout-B spectrum: X[k1 + E k2] (k1 = l P + t) is kept at position
// E k2 + L t + l, so the L lanes of a transform store and load consecutive entries.
template <int N>
__device__ __forceinline__ int bpos(int lane, int t, int k2) {
  constexpr int L = Split<N>::L, E = Split<N>::E;
  return E * k2 + L * t + lane;
}
// Frequency index stored at position p of that order.
template <int N>
__device__ __forceinline__ int bfreq(int p) {
  constexpr int L = Split<N>::L, E = Split<N>::E, P = E / L;
  return (p % L) * P + (p % E) / L + E * (p / E);
}

template <typename T, int DIR, int TWS>
__device__ __forceinline__ cplx<T> twid(const cplx<T>* tw, int m) {
  cplx<T> w = tw[m * TWS];
  if (DIR > 0) w.im = -w.im;
  return w;
}

// Twiddles of the four-step split: twl[k1 * L + l] = exp(-2 pi i l k1 / N), laid out so the L
// lanes of a transform read consecutive entries.
template <typename T, int N>
__device__ __forceinline__ void fill_twl(cplx<T>* twl, const cplx<T>* tw2n, int tid, int nthreads) {
  constexpr int L = Split<N>::L, E = Split<N>::E;
  for (int i = tid; i < L * E; i += nthreads) {
    const int k1 = i / L, l = i - k1 * L;
    twl[i] = tw2n[2 * l * k1];
  }
}

template <typename T, int DIR>
__device__ __forceinline__ cplx<T> twl_get(const cplx<T>* twl, int i) {
  cplx<T> w = twl[i];
  if (DIR > 0) w.im = -w.im;
  return w;
}

template <typename T, int N, int DIR, int TWS>
__device__ __forceinline__ void fft_a2b(cplx<T> (&a)[Split<N>::E], cplx<T>* buf, int s, int lane, const cplx<T>* twl) {
  constexpr int L = Split<N>::L, E = Split<N>::E, P = E / L;
  SmallDFT<E, DIR, T>::run(a);
  if constexpr (L > 1) {
#pragma unroll
    for (int k1 = 1; k1 < E; ++k1) a[k1] = a[k1] * twl_get<T, DIR>(twl, k1 * L + lane);
    wave_sync();
#pragma unroll
    for (int k1 = 0; k1 < E; ++k1) buf[tpos<N>(k1, lane) * s] = a[k1];
    wave_sync();
#pragma unroll
    for (int t = 0; t < P; ++t)
#pragma unroll
      for (int m = 0; m < L; ++m) a[t * L + m] = buf[tpos<N>(lane * P + t, m) * s];
#pragma unroll
    for (int t = 0; t < P; ++t) SmallDFT<L, DIR, T>::run(&a[t * L]);
  }
}

template <typename T, int N, int DIR, int TWS>
__device__ __forceinline__ void fft_b2a(cplx<T> (&a)[Split<N>::E], cplx<T>* buf, int s, int lane, const cplx<T>* twl) {
  constexpr int L = Split<N>::L, E = Split<N>::E, P = E / L;
  if constexpr (L > 1) {
#pragma unroll
    for (int t = 0; t < P; ++t) SmallDFT<L, DIR, T>::run(&a[t * L]);
    wave_sync();
#pragma unroll
    for (int t = 0; t < P; ++t)
#pragma unroll
      for (int m = 0; m < L; ++m) buf[tpos<N>(lane * P + t, m) * s] = a[t * L + m];
    wave_sync();
#pragma unroll
    for (int k1 = 0; k1 < E; ++k1) a[k1] = buf[tpos<N>(k1, lane) * s];
#pragma unroll
    for (int k1 = 1; k1 < E; ++k1) a[k1] = a[k1] * twl_get<T, DIR>(twl, k1 * L + lane);
  }
  SmallDFT<E, DIR, T>::run(a);
}

// R rows at once: the same four-step transforms for R independent rows of one lane group, each
// row stored at stride 1 from rows[r] (its own scratch).  Interleaving the rows between the fences
// gives the wavefront R independent chains to overlap LDS latency with.
// rows_a2b: layout-A registers -> spectrum stored in bpos() order in each row.
template <typename T, int N, int DIR, int R>
__device__ __forceinline__ void rows_a2b(cplx<T> (&a)[R][Split<N>::E], cplx<T>* const (&rows)[R], int lane,
                                         const cplx<T>* twl) {
  constexpr int L = Split<N>::L, E = Split<N>::E, P = E / L;
#pragma unroll
  for (int r = 0; r < R; ++r) SmallDFT<E, DIR, T>::run(a[r]);
  if constexpr (L > 1) {
#pragma unroll
    for (int k1 = 1; k1 < E; ++k1) {
      const cplx<T> w = twl_get<T, DIR>(twl, k1 * L + lane);
#pragma unroll
      for (int r = 0; r < R; ++r) a[r][k1] = a[r][k1] * w;
    }
    wave_sync();
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int k1 = 0; k1 < E; ++k1) rows[r][tpos<N>(k1, lane)] = a[r][k1];
    wave_sync();
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int t = 0; t < P; ++t)
#pragma unroll
        for (int m = 0; m < L; ++m) a[r][t * L + m] = rows[r][tpos<N>(lane * P + t, m)];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int t = 0; t < P; ++t) SmallDFT<L, DIR, T>::run(&a[r][t * L]);
  }
  wave_sync();
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int t = 0; t < P; ++t)
#pragma unroll
      for (int k2 = 0; k2 < L; ++k2) rows[r][bpos<N>(lane, t, k2)] = a[r][t * L + k2];
  wave_sync();
}

// rows_b2a: spectrum in bpos() order in each row -> layout-A registers (the rows are scratch).
template <typename T, int N, int DIR, int R>
__device__ __forceinline__ void rows_b2a(cplx<T> (&a)[R][Split<N>::E], cplx<T>* const (&rows)[R], int lane,
                                         const cplx<T>* twl) {
  constexpr int L = Split<N>::L, E = Split<N>::E, P = E / L;
  wave_sync();
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int t = 0; t < P; ++t)
#pragma unroll
      for (int k2 = 0; k2 < L; ++k2) a[r][t * L + k2] = rows[r][bpos<N>(lane, t, k2)];
  if constexpr (L > 1) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int t = 0; t < P; ++t) SmallDFT<L, DIR, T>::run(&a[r][t * L]);
    wave_sync();
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int t = 0; t < P; ++t)
#pragma unroll
        for (int m = 0; m < L; ++m) rows[r][tpos<N>(lane * P + t, m)] = a[r][t * L + m];
    wave_sync();
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int k1 = 0; k1 < E; ++k1) a[r][k1] = rows[r][tpos<N>(k1, lane)];
#pragma unroll
    for (int k1 = 1; k1 < E; ++k1) {
      const cplx<T> w = twl_get<T, DIR>(twl, k1 * L + lane);
#pragma unroll
      for (int r = 0; r < R; ++r) a[r][k1] = a[r][k1] * w;
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) SmallDFT<E, DIR, T>::run(a[r]);
  wave_sync();
}

}  // namespace ls
