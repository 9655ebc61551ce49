// Hot-path kernels of the Lippmann-Schwinger forward model on gfx950.
//
// The volume operator G of Proposition 2 is a linear convolution of an n^3 field with the
// modified kernel gm on the 2n grid, i.e. (G v) = crop(F^{-1}_{2n}(ghat_m . F_{2n}(pad v))).
// Splitting every 2n-point axis transform into its even and odd output frequencies turns the
// zero-padded 2n-point DFT into two n-point DFTs (the odd one of the input modulated by
// exp(-i pi j / n)), and the cropped inverse into the sum of two n-point inverse DFTs.  The
// convolution is evaluated in three passes over HBM:
//
//   k_xfwd  [z][y][x] field -> x-spectrum [kx (2n)][z][y]           (prologue fuses f . x and
//                                                                      the Krylov vector updates)
//   k_yzc   per (slot, kx, ky class): padded y-DFT of one class of C (ky = c mod C) as a
//   k_yz3   2n/C-point DFT of the folded row, z-convolution with ghat_m, inverse, written
//           class-major [c][kx][z][j] (k_yz3: C = 2, the parity split)
//   k_xinv  class sum, cropped inverse x-DFT -> [z][y][x]              (epilogue fuses x - G(...)
//                                                                      and FP64 partial dots)
//
// The far field (eq. (lipp2), P = I) reuses k_xfwd/k_xinv with k_ff / k_ffT in between.
// Kernels of the Fourier-domain Green function carry the 1/(2n)^d normalisation of the inverse
// transforms, so every FFT here is unnormalised.
#include "fft.hpp"
#include "launch.hpp"


namespace ls {

// Device-memory accessors.  Slot vectors are reached through descriptor pointers, which the
// compiler cannot prove global; the casts make it emit global (not flat) memory instructions,
// so LDS waits inside the transforms do not also wait for outstanding HBM loads.
#define LS_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ cplx<T> ld(const void* p, size_t i) {
  const LS_GLOBAL T* q = (const LS_GLOBAL T*)p;
  return cplx<T>{q[2 * i], q[2 * i + 1]};
}
// Nontemporal load of a streamed field: the solver vectors are each read once per pass, so they
// are not kept in the caches (measured 4-8 % faster for the x-forward pass and the update).
template <typename T>
__device__ __forceinline__ cplx<T> ldn(const void* p, size_t i) {
  const LS_GLOBAL T* q = (const LS_GLOBAL T*)p;
  return cplx<T>{__builtin_nontemporal_load(&q[2 * i]), __builtin_nontemporal_load(&q[2 * i + 1])};
}
// Stores are nontemporal: every field a pass writes is read back by a later pass only after far
// more data than the caches hold has streamed through (measured 2-7 % faster per pass).
template <typename T>
__device__ __forceinline__ void stv(void* p, size_t i, cplx<T> v) {
  LS_GLOBAL T* q = (LS_GLOBAL T*)p;
  __builtin_nontemporal_store(v.re, &q[2 * i]);
  __builtin_nontemporal_store(v.im, &q[2 * i + 1]);
}
template <typename T>
__device__ __forceinline__ T ldr(const void* p, size_t i) { return ((const LS_GLOBAL T*)p)[i]; }
// Load at a 32-bit byte offset from a base that is uniform across the wavefront: the address
// is formed by the memory instruction (scalar base + vector offset), with no 64-bit vector
// arithmetic per load.
template <typename T>
__device__ __forceinline__ cplx<T> ldo(const void* base, uint32_t boff) {
  const LS_GLOBAL T* q = (const LS_GLOBAL T*)((const LS_GLOBAL char*)base + boff);
  return cplx<T>{q[0], q[1]};
}

__device__ __forceinline__ bool slot_active(const PassArgs& a, int slot) {
  return (a.mask >> a.st[slot].status) & 1u;
}

// Plane wave exp(i k d.x), x = signed voxel position (index - n/2 + 1).  The phase is formed
// in FP64 and reduced to [-pi, pi] before a single-precision sincos on the c64 path.
template <typename T>
__device__ __forceinline__ cplx<T> plane_wave(const SlotDesc& d, int n, int z, int y, int x) {
  const double c0 = 1.0 - 0.5 * n;
  const double ph = d.k * (d.d[0] * (x + c0) + d.d[1] * (y + c0) + d.d[2] * (z + c0));
  if constexpr (std::is_same<T, double>::value) {
    double s, c;
    sincos(ph, &s, &c);
    return {c, s};
  } else {
    const double r = ph - 6.283185307179586477 * rint(ph * 0.15915494309189533577);
    float s, c;
    sincosf((float)r, &s, &c);
    return {c, s};
  }
}

template <typename T>
__device__ __forceinline__ cplx<T> rhs_b(const SlotDesc& d, int n, size_t idx, int z, int y, int x) {
  if (d.vec[V_B]) return ldn<T>(d.vec[V_B], idx);
  return plane_wave<T>(d, n, z, y, x);
}

template <typename T>
__device__ __forceinline__ cplx<T> scal(const double* v) { return {(T)v[0], (T)v[1]}; }

__device__ __forceinline__ double* part_ptr(const PassArgs& a, int slot, int blk, int j) {
  return a.part + (((size_t)slot * a.part_stride + blk) * PART_K + j) * 2;
}

// =============================================================================================
// Row transforms of length N held in LDS (stride 1), by L lanes: natural-order signal, spectrum in
// the storage order of bpos() (natural order for the Stockham sizes).
template <int N>
struct HasSplit {
  static constexpr bool value = (N == 8 || N == 16 || N == 32 || N == 48 || N == 64 || N == 96 || N == 128 ||
                                 N == 192 || N == 256);
};

template <typename T, int N, int DIR, int TWS = 2>
__device__ __forceinline__ void row_fft(cplx<T>* row, int lane, const cplx<T>* tw, const cplx<T>* twl) {
  if constexpr (HasSplit<N>::value) {
    constexpr int L = Split<N>::L, E = Split<N>::E, P = E / L;
    cplx<T> v[E];
    if (DIR < 0) {
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = row[lane + L * j];
      fft_a2b<T, N, DIR, 2>(v, row, 1, lane, twl);
      wave_sync();
#pragma unroll
      for (int t = 0; t < P; ++t)
#pragma unroll
        for (int k2 = 0; k2 < L; ++k2) row[bpos<N>(lane, t, k2)] = v[t * L + k2];
    } else {
#pragma unroll
      for (int t = 0; t < P; ++t)
#pragma unroll
        for (int k2 = 0; k2 < L; ++k2) v[t * L + k2] = row[bpos<N>(lane, t, k2)];
      fft_b2a<T, N, DIR, 2>(v, row, 1, lane, twl);
      wave_sync();
#pragma unroll
      for (int j = 0; j < E; ++j) row[lane + L * j] = v[j];
    }
    wave_sync();
  } else {
    fft_group<T, N, DIR, TWS>(row, 1, lane, tw);
  }
}

template <int N>
constexpr int twl_size() {
  if constexpr (HasSplit<N>::value)
    return N;
  else
    return 1;
}

template <typename T, int N>
__device__ __forceinline__ void fill_twl_any(cplx<T>* twl, const cplx<T>* tw, int tid, int nt) {
  if constexpr (HasSplit<N>::value) fill_twl<T, N>(twl, tw, tid, nt);
}

// Position of frequency k in a row spectrum produced by row_fft.
template <int N>
__device__ __forceinline__ int spec_pos(int k) {
  if constexpr (HasSplit<N>::value) {
    constexpr int L = Split<N>::L, E = Split<N>::E, P = E / L;
    return E * (k / E) + L * ((k % E) % P) + (k % E) / P;
  } else {
    return k;
  }
}
template <int N>
__device__ __forceinline__ int spec_freq(int p) {
  if constexpr (HasSplit<N>::value)
    return bfreq<N>(p);
  else
    return p;
}

// Lane groups of one wavefront take rows (or columns) L apart: with a pitch of N + 1 complex the
// accesses of consecutive groups then land on disjoint LDS banks.
template <int N, int L>
__device__ __forceinline__ int spreadL(int idx) {
  return L * (idx % (N / L)) + idx / (N / L);
}

template <int N>
constexpr int row_lanes() {
  if constexpr (HasSplit<N>::value)
    return Split<N>::L;
  else
    return Lanes<N>::value;
}

constexpr int largest_divisor_upto(int n, int cap) {
  int d = cap < n ? cap : n;
  while (n % d) --d;
  return d;
}

template <int N>
struct XCfg {
  static constexpr int TY = N < 16 ? N : 16;
  static constexpr int NYT = N / TY;
  static constexpr int PITCH = N + 1;
  static constexpr int IT = (TY * N + 255) / 256;       // elements per thread, [y][x] tile
  static constexpr int IT2 = (2 * N * TY + 255) / 256;  // elements per thread, [kx][y] tile
};

// Block order of the x-forward pass, by measurement (60-slot launches, all slots active):
// slot-major in launch order (round robin over the XCDs), or XCD-aware, each XCD taking one
// contiguous run of slots and tiles.  The latter is 2-16 % faster from n = 96 up (256^3 complex64:
// 8.13 against 9.65 ms, 5.95 TB/s; complex128 at 128: 1.94 against 2.27 ms), but 5 % slower at
// n <= 64 and 2 % slower for complex64 at 128, which keep launch order.  (An order with the slot
// fastest, so that the f tile stays in L2 across slots, varied from 1.02 to 1.28 ms at 128^3
// with where the slot fields sit in memory; f's re-reads are mostly served before HBM anyway.)
template <typename T, int N>
constexpr bool xfwd_xcd_order() {
  return N >= 96 && !(sizeof(T) == 4 && N == 128);
}

// =============================================================================================
// k_xfwd: prologue, zero-extension n -> 2n along x and the two n-point x-DFTs of each row.
// Every global load of a thread is issued before the first use (unrolled), so the loads of a
// wavefront overlap instead of paying the memory latency one at a time.
template <typename T, int N, int MODE>
__global__ __launch_bounds__(256) void k_xfwd(PassArgs a) {
  using X = XCfg<N>;
  constexpr int TY = X::TY, NYT = X::NYT, PITCH = X::PITCH, IT = X::IT, IT2 = X::IT2;
  constexpr int L = row_lanes<N>();
  constexpr int NG = 256 / L;
  __shared__ cplx<T> bufE[TY * PITCH];
  __shared__ cplx<T> bufO[TY * PITCH];
  __shared__ cplx<T> tw[2 * N];
  __shared__ cplx<T> twl[twl_size<N>()];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int lin = (xfwd_xcd_order<T, N>() && nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int per = a.nz * NYT;
  const int slot = lin / per;
  const int blk = lin - slot * per;
  if (!slot_active(a, slot)) return;
  const int z = blk / NYT;
  const int y0 = (blk - z * NYT) * TY;
  const SlotDesc& d = a.desc[slot];
  const SlotState& st = a.st[slot];
  if constexpr (MODE == PRO_F_B) {
    // the initial-residual pass is a slot's first work: its start time on the device clock
    if (blk == 0 && tid == 0) a.st[slot].t_start = (uint64_t)wall_clock64();
  }
  for (int i = tid; i < 2 * N; i += 256) tw[i] = ld<T>(a.tw, i);

  const size_t row0 = ((size_t)z * N + y0) * N;
  constexpr bool HAS_F = !(MODE == PRO_VEC || MODE == PRO_CONJ_VEC);
  cplx<T> r0[IT], r1[IT], r2[IT];
  T ff[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int i = tid + it * 256;
    if (i < TY * N) {
      const size_t idx = row0 + i;
      if constexpr (MODE == PRO_F_VEC || MODE == PRO_VEC || MODE == PRO_CONJ_VEC) r0[it] = ldn<T>(d.vec[a.sel], idx);
      if constexpr (MODE == PRO_P || MODE == PRO_S) {
        r0[it] = ldn<T>(d.vec[V_R], idx);
        r2[it] = ldn<T>(d.vec[V_V], idx);
      }
      if constexpr (MODE == PRO_P) r1[it] = ldn<T>(d.vec[V_P], idx);
      if constexpr (MODE == PRO_F_B) {
        if (d.vec[V_B]) r0[it] = ldn<T>(d.vec[V_B], idx);
      }
      if constexpr (HAS_F) ff[it] = ldr<T>(d.f, idx);
    }
  }
  const cplx<T> alpha = scal<T>(st.alpha), beta = scal<T>(st.beta), omega = scal<T>(st.omega);
  const bool restart = st.restart_flag != 0;
  double ss = 0.0;
  __syncthreads();
  fill_twl_any<T, N>(twl, tw, tid, 256);
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int i = tid + it * 256;
    if (i < TY * N) {
      const int yy = i / N;
      const int x = i - yy * N;
      const size_t idx = row0 + i;
      cplx<T> w;
      if constexpr (MODE == PRO_F_VEC) {
        w = ff[it] * r0[it];
      } else if constexpr (MODE == PRO_F_B) {
        w = ff[it] * (d.vec[V_B] ? r0[it] : plane_wave<T>(d, N, z, y0 + yy, x));
      } else if constexpr (MODE == PRO_P) {
        cplx<T> p;
        if (restart) {
          p = r0[it];
          stv<T>(d.vec[V_RH], idx, p);
        } else {
          p = r0[it] + beta * (r1[it] - omega * r2[it]);
        }
        stv<T>(d.vec[V_P], idx, p);
        w = ff[it] * p;
      } else if constexpr (MODE == PRO_S) {
        const cplx<T> sv = r0[it] - alpha * r2[it];
        stv<T>(d.vec[V_S], idx, sv);
        ss += (double)sv.re * sv.re + (double)sv.im * sv.im;
        w = ff[it] * sv;
      } else if constexpr (MODE == PRO_VEC) {
        w = r0[it];
      } else {
        w = conj(r0[it]);
      }
      bufE[yy * PITCH + x] = w;
      bufO[yy * PITCH + x] = w * tw[x];
    }
  }
  __syncthreads();
  {
    const int g = tid / L, lane = tid - (tid / L) * L;
    for (int u = g; u < 2 * TY; u += NG) {
      const int t = (u % 4) * (2 * TY / 4) + u / 4;
      cplx<T>* base = t < TY ? bufE + t * PITCH : bufO + (t - TY) * PITCH;
      row_fft<T, N, -1>(base, lane, tw, twl);
    }
  }
  __syncthreads();
  void* spec = d.vec[a.spec];
#pragma unroll
  for (int it = 0; it < IT2; ++it) {
    const int i = tid + it * 256;
    if (i < 2 * N * TY) {
      const int yy = i % TY;
      const int kx = i / TY;
      const cplx<T>* src = (kx & 1) ? bufO : bufE;
      stv<T>(spec, ((size_t)kx * a.nz + z) * N + y0 + yy, src[yy * PITCH + spec_pos<N>(kx >> 1)]);
    }
  }
  if constexpr (MODE == PRO_S) {
    double v[1] = {ss};
    block_sum<1>(v, red);
    if (tid == 0) {
      double* pp = part_ptr(a, slot, blk, 0);
      pp[0] = v[0];
      pp[1] = 0.0;
    }
  }
}

// =============================================================================================
// k_xinv: inverse x-DFTs (even + modulated odd half), crop to n, epilogue and FP64 partials.
// Threads per workgroup: complex64 tiles (2 x 16 rows of n + 1 values) above 56 KB leave room for
// two workgroups per CU only, so they get 512 threads (16 waves per CU instead of 8 keep more
// loads in flight) with registers for 4 waves per SIMD; complex128 keeps 256 threads (its
// register sets would spill at that occupancy).
template <typename T, int N>
struct XInvCfg {
  static constexpr bool WIDE = sizeof(T) == 4 && 2 * XCfg<N>::TY * XCfg<N>::PITCH * (int)sizeof(cplx<T>) > 56 * 1024;
  static constexpr int NT = WIDE ? 512 : 256;
  static constexpr int WPE = WIDE ? 4 : 1;
  // class sum by a C-point DFT over the classes: a tile holds TY / (C/2) consecutive j of every
  // period y = j + k 2n/C, k < C/2, so each class value is loaded once and gives the C/2 rows that
  // share it.  It pays for the wide complex64 tiles (n = 256, eight classes: 6 % less time than
  // Horner's rule); at n = 128 the extra registers of the C values per output cost more than the
  // repeated class loads (which L2 serves) save, in either precision.
  static constexpr bool DFTSUM = WIDE;
  // whether the class sum of CL classes takes the DFT form; the plane pass then writes the classes
  // z-major, [c][z][kx][j], so that the rows one tile reads per class lie in one 2n CM block
  // instead of 2n lines a whole kx plane apart (measured kx-major at 256^3: the L2 fetched each
  // of those lines about 1.8 times before the neighbouring tiles had read the rest of it)
  static constexpr bool dftsum(int CL) {
    return DFTSUM && (CL == 4 || CL == 8) && XCfg<N>::TY % (CL / 2) == 0 &&
           (2 * N / CL) % (2 * XCfg<N>::TY / CL) == 0 && (2 * N / CL) / (2 * XCfg<N>::TY / CL) == XCfg<N>::NYT;
  }
  static constexpr int IT = (XCfg<N>::TY * N + NT - 1) / NT;
  static constexpr int IT2 = (2 * N * XCfg<N>::TY + NT - 1) / NT;
  // outputs per thread handled in one chunk of the class sum (three chunk-sized register sets)
  static constexpr int ITC_MAX = WIDE ? 8 : (sizeof(T) == 4 ? 16 : 8);
};

template <typename T, int N, int EPI, int CL>
__global__ __launch_bounds__((XInvCfg<T, N>::NT), (XInvCfg<T, N>::WPE)) void k_xinv(PassArgs a) {
  using X = XCfg<N>;
  using XI = XInvCfg<T, N>;
  constexpr int NTX = XI::NT;
  constexpr int TY = X::TY, NYT = X::NYT, PITCH = X::PITCH, IT = XI::IT, IT2 = XI::IT2;
  constexpr int L = row_lanes<N>();
  constexpr int NG = NTX / L;
  __shared__ cplx<T> bufE[TY * PITCH];
  __shared__ cplx<T> bufO[TY * PITCH];
  __shared__ cplx<T> tw[2 * N];
  __shared__ cplx<T> twl[twl_size<N>()];
  __shared__ double red[6 * (NTX / 64)];
  const int tid = threadIdx.x;
  // CL = 1: plain x-spectrum [kx][z][y].  CL > 1: class-major output of the (y,z) pass,
  // [c][kx][z][j] with rows of CM = 2n / CL (periodic in y with period CM); the value at y is
  // sum_c exp(+i pi c y / n) Y_c[y mod CM].
  constexpr int CM = CL == 1 ? N : 2 * N / CL;
  constexpr int TPP = CM / TY;   // y tiles per period
  constexpr int FA = NYT / TPP;  // periods per row: tiles reading the same class rows
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  // consecutive blocks on one XCD are the FA tiles of one (slot, z) that read the same class
  // values, so all but the first find them in L2.  Each XCD takes one eighth of the z range for
  // every slot (runs of consecutive z per slot), so a launch with few active slots still uses
  // all XCDs.
  const int lin = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int zs = lin / NYT;
  const int tr = lin - zs * NYT;
  const int ZB = (a.nz % 8 == 0) ? a.nz / 8 : 1;
  const int zb = zs / (a.nslots * ZB);
  const int rem = zs - zb * a.nslots * ZB;
  const int slot = rem / ZB;
  const int z = zb * ZB + (rem - slot * ZB);
  if (!slot_active(a, slot)) return;
  const int blk = z * NYT + tr;
  constexpr bool DS = XI::dftsum(CL);
  constexpr int KP = DS ? CL / 2 : 1;   // periods per tile (DFTSUM)
  constexpr int TYJ = TY / KP;          // consecutive j per period (DFTSUM)
  const int y0 = DS ? tr * TYJ : ((tr / FA) + (tr % FA) * TPP) * TY;
  // global y of tile row yy: TY consecutive rows, or (DFTSUM) KP runs of TYJ rows, CM apart
  auto yrow = [&](int yy) { return DS ? y0 + yy % TYJ + (yy / TYJ) * CM : y0 + yy; };
  const SlotDesc& d = a.desc[slot];
  for (int i = tid; i < 2 * N; i += NTX) tw[i] = ld<T>(a.tw, i);
  if constexpr (DS) {
    static_assert(TY % KP == 0 && CM % TYJ == 0 && CM / TYJ == NYT, "DFT class-sum tiles");
    // thread -> (kx, jj); per kx and class one TYJ-long row piece of the z-major class array
    const void* spec = d.vec[a.spec];
    const size_t cstride = (size_t)2 * N * a.nz * CM * sizeof(cplx<T>);
    constexpr int PAIRS = 2 * N * TYJ;
    constexpr int PT = PAIRS / NTX;       // pairs per thread
    static_assert(PAIRS % NTX == 0, "pairs per thread");
    cplx<T> v[PT][CL];
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      const int pidx = tid + q * NTX;
      const int kx = pidx / TYJ, jj = pidx - (pidx / TYJ) * TYJ;
      const uint32_t off = (uint32_t)((z * 2 * N + kx) * CM + y0 + jj) * (uint32_t)sizeof(cplx<T>);
#pragma unroll
      for (int c = 0; c < CL; ++c) v[q][c] = ldo<T>((const char*)spec + (size_t)c * cstride, off);
    }
    __syncthreads();  // tw visible
    fill_twl_any<T, N>(twl, tw, tid, NTX);
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      const int pidx = tid + q * NTX;
      const int kx = pidx / TYJ, jj = pidx - (pidx / TYJ) * TYJ;
      const int j = y0 + jj;
      // z_c = exp(+i pi c j / n) Y_c, then Y(j + k CM) = sum_c z_c exp(+2 pi i c k / C), k < C/2
#pragma unroll
      for (int c = 1; c < CL; ++c) v[q][c] = mulc(v[q][c], tw[(c * j) % (2 * N)]);
      SmallDFT<CL, +1, T>::run(v[q]);
      cplx<T>* buf = (kx & 1) ? bufO : bufE;
#pragma unroll
      for (int k = 0; k < KP; ++k) buf[(k * TYJ + jj) * PITCH + spec_pos<N>(kx >> 1)] = v[q][k];
    }
  } else {
    static_assert(CL == 1 || (CM % TY == 0 && CL % 2 == 0), "y tiles must stay inside one period");
    const void* spec = d.vec[a.spec];
    const int j0 = y0 % CM;
    // byte offset of (kx, z, j0 + yy) inside one class block; class blocks are 2n nz CM apart
    const size_t cstride = (size_t)2 * N * a.nz * CM * sizeof(cplx<T>);
    const uint32_t off0 = (uint32_t)(((tid / TY) * a.nz + z) * CM + j0 + tid % TY) * (uint32_t)sizeof(cplx<T>);
    constexpr uint32_t OFF_IT = (NTX / TY) * CM * sizeof(cplx<T>);  // per it: NTX / TY more kx
    // outputs are handled in chunks of ITC per thread so that three chunk-sized register sets
    // (sum, current class, next class) fit beside the rest of the kernel
    constexpr int ITC = largest_divisor_upto(IT2, XI::ITC_MAX);
    auto load = [&](cplx<T>(&v)[ITC], int c, int it0) {
      const char* cbase = (const char*)spec + (size_t)c * cstride;
#pragma unroll
      for (int k = 0; k < ITC; ++k) {
        const int it = it0 + k;
        const int i = tid + it * NTX;
        if (i < 2 * N * TY) v[k] = ldo<T>(cbase, off0 + (uint32_t)it * OFF_IT * (uint32_t)a.nz);
      }
    };
    // sum_c w^c Y_c with w = exp(+i pi y / n), by Horner's rule from the last class down; the
    // loads of the next class are in flight while the current one is accumulated
#pragma unroll 1
    for (int it0 = 0; it0 < IT2; it0 += ITC) {
      cplx<T> acc[ITC];
      if constexpr (CL == 1) {
        load(acc, 0, it0);
        if (it0 == 0) {
          __syncthreads();  // tw visible
          fill_twl_any<T, N>(twl, tw, tid, NTX);
        }
      } else {
        cplx<T> va[ITC], vb[ITC];
        load(va, CL - 1, it0);
        load(vb, CL - 2, it0);
        if (it0 == 0) {
          __syncthreads();  // tw visible
          fill_twl_any<T, N>(twl, tw, tid, NTX);
        }
        const cplx<T> wy = conj(tw[y0 + tid % TY]);
#pragma unroll
        for (int k = 0; k < ITC; ++k) acc[k] = va[k];
#pragma unroll 1
        for (int c = CL - 2; c >= 2; c -= 2) {
          load(va, c - 1, it0);
#pragma unroll
          for (int k = 0; k < ITC; ++k) acc[k] = acc[k] * wy + vb[k];
          load(vb, c - 2, it0);
#pragma unroll
          for (int k = 0; k < ITC; ++k) acc[k] = acc[k] * wy + va[k];
        }
#pragma unroll
        for (int k = 0; k < ITC; ++k) acc[k] = acc[k] * wy + vb[k];
      }
#pragma unroll
      for (int k = 0; k < ITC; ++k) {
        const int i = tid + (it0 + k) * NTX;
        if (i < 2 * N * TY) {
          const int yy = i % TY;
          const int kx = i / TY;
          ((kx & 1) ? bufO : bufE)[yy * PITCH + spec_pos<N>(kx >> 1)] = acc[k];
        }
      }
    }
  }
  __syncthreads();
  {
    const int g = tid / L, lane = tid - (tid / L) * L;
    for (int u = g; u < 2 * TY; u += NG) {
      const int t = (u % 4) * (2 * TY / 4) + u / 4;
      cplx<T>* base = t < TY ? bufE + t * PITCH : bufO + (t - TY) * PITCH;
      row_fft<T, N, +1>(base, lane, tw, twl);
    }
  }
  __syncthreads();
  cplx<T> q0[IT], q1[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int i = tid + it * NTX;
    if (i < TY * N) {
      const size_t idx = ((size_t)z * N + yrow(i / N)) * N + i % N;
      if constexpr (EPI == EPI_AXV) {
        q0[it] = ldn<T>(d.vec[V_P], idx);
        q1[it] = ldn<T>(d.vec[V_RH], idx);
      } else if constexpr (EPI == EPI_AXT) {
        q0[it] = ldn<T>(d.vec[V_S], idx);
      } else if constexpr (EPI == EPI_R0) {
        if (d.vec[V_B]) q0[it] = ldn<T>(d.vec[V_B], idx);
      } else if constexpr (EPI == EPI_TRUE || EPI == EPI_R0X) {
        if (d.vec[V_B]) q0[it] = ldn<T>(d.vec[V_B], idx);
        q1[it] = ldn<T>(d.vec[V_X], idx);
      } else if constexpr (EPI == EPI_AX) {
        q0[it] = ldn<T>(d.vec[a.sel], idx);
      }
    }
  }
  cplx<double> a0 = {0, 0}, a1 = {0, 0}, a2 = {0, 0};
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int i = tid + it * NTX;
    if (i < TY * N) {
      const int yy = i / N;
      const int x = i - yy * N;
      const size_t idx = ((size_t)z * N + yrow(yy)) * N + x;
      const cplx<T> g = bufE[yy * PITCH + x] + mulc(bufO[yy * PITCH + x], tw[x]);
      if constexpr (EPI == EPI_STORE) {
        stv<T>(d.vec[a.sel], idx, g);
      } else if constexpr (EPI == EPI_AXV) {
        const cplx<T> v = q0[it] - g;
        stv<T>(d.vec[V_V], idx, v);
        dot_acc(a0, q1[it], v);
      } else if constexpr (EPI == EPI_AXT) {
        const cplx<T> t = q0[it] - g;
        stv<T>(d.vec[V_T], idx, t);
        dot_acc(a1, t, q0[it]);
        a2.re += (double)t.re * t.re + (double)t.im * t.im;
      } else if constexpr (EPI == EPI_R0) {
        const cplx<T> b = d.vec[V_B] ? q0[it] : plane_wave<T>(d, N, z, yrow(yy), x);
        stv<T>(d.vec[V_X], idx, b);
        stv<T>(d.vec[V_R], idx, g);
        stv<T>(d.vec[V_RH], idx, g);
        a0.re += (double)g.re * g.re + (double)g.im * g.im;
        a1.re += (double)b.re * b.re + (double)b.im * b.im;
      } else if constexpr (EPI == EPI_TRUE) {
        const cplx<T> b = d.vec[V_B] ? q0[it] : plane_wave<T>(d, N, z, yrow(yy), x);
        const cplx<T> r = (b - q1[it]) + g;
        stv<T>(d.vec[V_R], idx, r);
        a0.re += (double)r.re * r.re + (double)r.im * r.im;
      } else if constexpr (EPI == EPI_R0X) {
        const cplx<T> b = d.vec[V_B] ? q0[it] : plane_wave<T>(d, N, z, yrow(yy), x);
        const cplx<T> r = (b - q1[it]) + g;
        stv<T>(d.vec[V_R], idx, r);
        stv<T>(d.vec[V_RH], idx, r);
        a0.re += (double)r.re * r.re + (double)r.im * r.im;
        a1.re += (double)b.re * b.re + (double)b.im * b.im;
      } else {  // EPI_AX
        stv<T>(d.vec[a.sel2], idx, q0[it] - g);
      }
    }
  }
  if constexpr (EPI == EPI_AXV || EPI == EPI_AXT || EPI == EPI_R0 || EPI == EPI_R0X || EPI == EPI_TRUE) {
    double v[6] = {a0.re, a0.im, a1.re, a1.im, a2.re, a2.im};
    block_sum<6>(v, red);
    if (tid == 0) {
      if constexpr (EPI == EPI_AXV || EPI == EPI_TRUE) {
        double* pp = part_ptr(a, slot, blk, 0);
        pp[0] = v[0];
        pp[1] = v[1];
      } else if constexpr (EPI == EPI_R0 || EPI == EPI_R0X) {
        double* pp = part_ptr(a, slot, blk, 0);
        pp[0] = v[0];
        pp[1] = 0.0;
        pp[2] = v[2];
        pp[3] = 0.0;
      } else {  // EPI_AXT: entries 1 and 2 (entry 0 holds ||s||^2 from k_xfwd)
        double* pp = part_ptr(a, slot, blk, 1);
        pp[0] = v[2];
        pp[1] = v[3];
        pp[2] = v[4];
        pp[3] = 0.0;
      }
    }
  }
}

// =============================================================================================
// Plane kernels: one workgroup per (slot, kx) plane of the x-spectrum, the whole n x n plane in
// LDS.  Blocks are numbered so that consecutive blocks on one XCD (workgroups go round-robin
// over the 8 XCDs) share kx and therefore the same kernel plane in that XCD's L2.
template <int N>
struct PlaneCfg {
  static constexpr int NT = N * N >= 16384 ? 1024 : (N * N >= 8192 ? 512 : (N * N >= 256 ? 256 : N * N));
  static constexpr int PER = N * N / NT;
  static constexpr int PITCH = N + 1;
  static_assert(PER * NT == N * N, "plane must split evenly over the block");
};

__device__ __forceinline__ void plane_decode(const PassArgs& a, int& kx, int& slot) {
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int lin = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  kx = lin / a.nslots;
  slot = lin - kx * a.nslots;
}

// z-convolution of one column (length N, stride `pitch` in LDS) with the kernel row
// krow[kz], kz in [0, 2N): the 2N-point zero-padded DFT is split into its even and odd output
// frequencies, each multiplied by its kernel samples and inverted, and the two halves recombined.
template <typename T, int N>
__device__ __forceinline__ void zconv(cplx<T>* col, int pitch, int lane, const cplx<T>* tw, const cplx<T>* krow) {
  constexpr int E = Plan<N>::E;
  constexpr int L = N / E;
  cplx<T> orig[E], ev[E];
  wave_sync();
#pragma unroll
  for (int e = 0; e < E; ++e) orig[e] = col[(lane + e * L) * pitch];
  fft_group<T, N, -1, 2>(col, pitch, lane, tw);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int m = lane + e * L;
    col[m * pitch] = col[m * pitch] * krow[2 * m];
  }
  fft_group<T, N, +1, 2>(col, pitch, lane, tw);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int zz = lane + e * L;
    ev[e] = col[zz * pitch];
    col[zz * pitch] = orig[e] * tw[zz];
  }
  fft_group<T, N, -1, 2>(col, pitch, lane, tw);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int m = lane + e * L;
    col[m * pitch] = col[m * pitch] * krow[2 * m + 1];
  }
  fft_group<T, N, +1, 2>(col, pitch, lane, tw);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int zz = lane + e * L;
    col[zz * pitch] = ev[e] + mulc(col[zz * pitch], tw[zz]);
  }
  wave_sync();
}

// z-convolution of one column with four-step transforms; the kernel coefficients of both
// z-parities are requested before the forward transform so their latency overlaps it.
template <typename T>
struct alignas(4 * sizeof(T)) cpair {
  cplx<T> a, b;
};

template <typename T, int N, int PITCH, bool LEAN = (Split<N>::E * sizeof(T) > 64)>
__device__ __forceinline__ void zconv4(cplx<T>* col, int lane, const cplx<T>* tw, const cplx<T>* twl,
                                       const cplx<T>* kr) {
  constexpr int L = Split<N>::L, E = Split<N>::E, P = E / L;
  const LS_GLOBAL T* k2p = (const LS_GLOBAL T*)kr;
  cplx<T> e[E], o[E];
  if constexpr (LEAN) {
    // register-lean order for long per-lane transforms: each parity's kernel samples are loaded
    // only once its forward transform is done
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int zz = lane + L * j;
      e[j] = col[zz * PITCH];
      o[j] = e[j] * tw[zz];
    }
    fft_a2b<T, N, -1, 2>(e, col, PITCH, lane, twl);
#pragma unroll
    for (int t = 0; t < P; ++t)
#pragma unroll
      for (int k2 = 0; k2 < L; ++k2) {
        const LS_GLOBAL T* q = k2p + 4 * (lane * P + t + E * k2);
        e[t * L + k2] = e[t * L + k2] * cplx<T>{q[0], q[1]};
      }
    fft_b2a<T, N, +1, 2>(e, col, PITCH, lane, twl);
    fft_a2b<T, N, -1, 2>(o, col, PITCH, lane, twl);
#pragma unroll
    for (int t = 0; t < P; ++t)
#pragma unroll
      for (int k2 = 0; k2 < L; ++k2) {
        const LS_GLOBAL T* q = k2p + 4 * (lane * P + t + E * k2);
        o[t * L + k2] = o[t * L + k2] * cplx<T>{q[2], q[3]};
      }
    fft_b2a<T, N, +1, 2>(o, col, PITCH, lane, twl);
    wave_sync();
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int zz = lane + L * j;
      col[zz * PITCH] = e[j] + mulc(o[j], tw[zz]);
    }
    return;
  }
  cpair<T> kk[E];
#pragma unroll
  for (int t = 0; t < P; ++t)
#pragma unroll
    for (int k2 = 0; k2 < L; ++k2) {
      const LS_GLOBAL T* q = k2p + 4 * (lane * P + t + E * k2);
      kk[t * L + k2] = cpair<T>{{q[0], q[1]}, {q[2], q[3]}};
    }
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int zz = lane + L * j;
    e[j] = col[zz * PITCH];
    o[j] = e[j] * tw[zz];
  }
  fft_a2b<T, N, -1, 2>(e, col, PITCH, lane, twl);
#pragma unroll
  for (int j = 0; j < E; ++j) e[j] = e[j] * kk[j].a;
  fft_b2a<T, N, +1, 2>(e, col, PITCH, lane, twl);
  fft_a2b<T, N, -1, 2>(o, col, PITCH, lane, twl);
#pragma unroll
  for (int j = 0; j < E; ++j) o[j] = o[j] * kk[j].b;
  fft_b2a<T, N, +1, 2>(o, col, PITCH, lane, twl);
  wave_sync();
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int zz = lane + L * j;
    col[zz * PITCH] = e[j] + mulc(o[j], tw[zz]);
  }
}

// k_yz3: one workgroup per (slot, kx, ky parity).  Reads the x-spectrum plane (modulated by
// exp(-i pi y / n) for the odd parity), y-DFT, z-convolution, inverse y-DFT, and writes the
// half to V_SPE / V_SPO; k_xinv adds the two halves.  Blocks are ordered (kx, slot, parity) per
// XCD so the two parity blocks of a plane follow each other (the second read of the plane hits
// L2) and all slots of one kx share the kernel plane in L2.
// LDS layout: plane rows have a pitch of N + 1 complex and the lane groups of a wavefront take
// rows / columns L apart, so row accesses, column accesses and the transposes of the four-step
// transforms spread over the banks; row spectra are kept in the order of bpos().
template <int N>
struct Plane3Cfg {
  static constexpr int NT = N >= 64 ? 512 : (N * N >= 256 ? 256 : N * N);
  static constexpr int PITCH = N + 1;
};

template <typename T, int N>
__global__ __launch_bounds__(Plane3Cfg<N>::NT) void k_yz3(PassArgs a) {
  constexpr int NT = Plane3Cfg<N>::NT, PITCH = Plane3Cfg<N>::PITCH;
  __shared__ cplx<T> plane[N * PITCH];
  __shared__ cplx<T> tw[2 * N];
  __shared__ cplx<T> twl[twl_size<N>()];
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int lin = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int par = lin & 1;
  const int ks = lin >> 1;
  const int kx = ks / a.nslots;
  const int slot = ks - kx * a.nslots;
  if (!slot_active(a, slot)) return;
  const int tid = threadIdx.x;
  const SlotDesc& d = a.desc[slot];
  const void* Sv = d.vec[a.spec];
  const size_t soff = (size_t)kx * N * N;
  void* Ov = d.vec[par ? V_SPO : V_SPE];
  const int kxp = kx <= N ? kx : 2 * N - kx;
  const cplx<T>* K = (const cplx<T>*)a.kern + (size_t)kxp * (4 * N * N);
  {
    constexpr int PER = N * N / NT;
    cplx<T> ldv[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) ldv[j] = ld<T>(Sv, soff + tid + j * NT);
    for (int i = tid; i < 2 * N; i += NT) tw[i] = ld<T>(a.tw, i);
    __syncthreads();
    fill_twl_any<T, N>(twl, tw, tid, NT);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int i = tid + j * NT;
      const int zz = i / N, y = i - zz * N;
      plane[zz * PITCH + y] = par ? ldv[j] * tw[y] : ldv[j];
    }
  }
  __syncthreads();
  if constexpr (!HasSplit<N>::value) {
    constexpr int L = Lanes<N>::value;
    constexpr int NG = NT / L;
    const int g = tid / L, lane = tid - g * L;
    for (int t = g; t < N; t += NG) fft_group<T, N, -1, 2>(plane + t * PITCH, 1, lane, tw);
    __syncthreads();
    for (int c = g; c < N; c += NG) zconv<T, N>(plane + c, PITCH, lane, tw, K + (size_t)(2 * c + par) * (2 * N));
    __syncthreads();
    for (int t = g; t < N; t += NG) fft_group<T, N, +1, 2>(plane + t * PITCH, 1, lane, tw);
  } else {
    constexpr int L = Split<N>::L;
    constexpr int G = NT / L;
    const int g = tid / L, lane = tid - g * L;
    for (int idx = g; idx < N; idx += G) row_fft<T, N, -1>(plane + spreadL<N, L>(idx) * PITCH, lane, tw, twl);
    __syncthreads();
    for (int idx = g; idx < N; idx += G) {
      const int c = spreadL<N, L>(idx);
      const int ky = spec_freq<N>(c);
      zconv4<T, N, PITCH>(plane + c, lane, tw, twl, K + (size_t)(2 * ky + par) * (2 * N));
    }
    __syncthreads();
    for (int idx = g; idx < N; idx += G) row_fft<T, N, +1>(plane + spreadL<N, L>(idx) * PITCH, lane, tw, twl);
  }
  __syncthreads();
  for (int i = tid; i < N * N; i += NT) {
    const int zz = i / N, y = i - zz * N;
    stv<T>(Ov, soff + i, plane[zz * PITCH + y]);
  }
}

// k_ff: far field, stage 2 of 3.  For one x-frequency plane of the spectrum of f.u:
// y-DFT of every z-row, multiply by the slice kernels Khat_z(kx, ky), sum over z, cropped
// inverse y-DFT.  Output [kx][y] (an x-spectrum with nz = 1) in vec[sel].
// Kernel layout: [kx' in 0..n][z in 0..n)[ky in 0..2n).
template <typename T, int N>
__global__ __launch_bounds__(PlaneCfg<N>::NT) void k_ff(PassArgs a) {
  using C = PlaneCfg<N>;
  constexpr int NT = C::NT, PER = C::PER, PITCH = C::PITCH;
  constexpr int L = Lanes<N>::value;
  constexpr int NG = NT / L;
  __shared__ cplx<T> plane[N * PITCH];
  __shared__ cplx<T> tw[2 * N];
  __shared__ cplx<T> yv[2 * N];
  int kx, slot;
  plane_decode(a, kx, slot);
  if (!slot_active(a, slot)) return;
  const int tid = threadIdx.x;
  const SlotDesc& d = a.desc[slot];
  for (int i = tid; i < 2 * N; i += NT) tw[i] = ld<T>(a.tw, i);
  const void* Sv = d.vec[a.spec];
  const size_t soff = (size_t)kx * N * N;
  const int kxp = kx <= N ? kx : 2 * N - kx;
  const cplx<T>* K = (const cplx<T>*)a.kern + (size_t)kxp * (2 * N * N);
  const int g = tid / L, lane = tid - (tid / L) * L;
  __syncthreads();
#pragma unroll 1
  for (int par = 0; par < 2; ++par) {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int i = tid + j * NT;
      const int zz = i / N, y = i - zz * N;
      cplx<T> v = ld<T>(Sv, soff + i);
      if (par) v = v * tw[y];
      plane[zz * PITCH + y] = v;
    }
    __syncthreads();
    for (int t = g; t < N; t += NG) fft_group<T, N, -1, 2>(plane + t * PITCH, 1, lane, tw);
    __syncthreads();
    // sum over z, split over ZS z-residues per ky so that every thread takes part; the partial
    // sums go to the first ZS plane rows once every thread is done reading the plane
    constexpr int ZS = NT / N >= 1 ? NT / N : 1;
    const int c = tid % N, zr = tid / N;
    cplx<T> acc = {0, 0};
    if (zr < ZS) {
      const cplx<T>* kz = K + 2 * c + par;
      for (int zz = zr; zz < N; zz += ZS) acc = acc + kz[(size_t)zz * 2 * N] * plane[zz * PITCH + c];
    }
    static_assert(NT >= N || ZS == 1, "one thread per ky at least");
    __syncthreads();
    if (zr < ZS) plane[zr * PITCH + c] = acc;
    __syncthreads();
    if (tid < N) {
      cplx<T> sum = plane[tid];
      for (int r = 1; r < ZS; ++r) sum = sum + plane[r * PITCH + tid];
      yv[par * N + tid] = sum;
    }
    __syncthreads();
  }
  if (g < 2) fft_group<T, N, +1, 2>(yv + g * N, 1, lane, tw);
  __syncthreads();
  cplx<T>* out = (cplx<T>*)d.vec[a.sel] + (size_t)kx * N;
  for (int y = tid; y < N; y += NT) out[y] = yv[y] + mulc(yv[N + y], tw[y]);
}

// k_ffT: transpose of the far field, stage 2 of 3.  Input: the x-spectrum [kx][y] (nz = 1) of a
// detector field in vec[sel].  For one kx: y-DFT of the row, multiply by every slice kernel,
// cropped inverse y-DFT of each z-row.  Output: x-spectrum plane [z][y] of vec[spec].
template <typename T, int N>
__global__ __launch_bounds__(PlaneCfg<N>::NT) void k_ffT(PassArgs a) {
  using C = PlaneCfg<N>;
  constexpr int NT = C::NT, PER = C::PER, PITCH = C::PITCH;
  constexpr int L = Lanes<N>::value;
  constexpr int NG = NT / L;
  __shared__ cplx<T> plane[N * PITCH];
  __shared__ cplx<T> tw[2 * N];
  __shared__ cplx<T> rv[2 * N];
  int kx, slot;
  plane_decode(a, kx, slot);
  if (!slot_active(a, slot)) return;
  const int tid = threadIdx.x;
  const SlotDesc& d = a.desc[slot];
  for (int i = tid; i < 2 * N; i += NT) tw[i] = ld<T>(a.tw, i);
  __syncthreads();
  const cplx<T>* row = (const cplx<T>*)d.vec[a.sel] + (size_t)kx * N;
  for (int y = tid; y < N; y += NT) {
    const cplx<T> v = row[y];
    rv[y] = v;
    rv[N + y] = v * tw[y];
  }
  const int g = tid / L, lane = tid - (tid / L) * L;
  __syncthreads();
  if (g < 2) fft_group<T, N, -1, 2>(rv + g * N, 1, lane, tw);
  __syncthreads();
  void* Sv = d.vec[a.spec];
  const size_t soff = (size_t)kx * N * N;
  const int kxp = kx <= N ? kx : 2 * N - kx;
  const cplx<T>* K = (const cplx<T>*)a.kern + (size_t)kxp * (2 * N * N);
  cplx<T> acc[PER];
#pragma unroll 1
  for (int par = 0; par < 2; ++par) {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int i = tid + j * NT;
      const int zz = i / N, c = i - zz * N;
      plane[zz * PITCH + c] = K[(size_t)zz * 2 * N + 2 * c + par] * rv[par * N + c];
    }
    __syncthreads();
    for (int t = g; t < N; t += NG) fft_group<T, N, +1, 2>(plane + t * PITCH, 1, lane, tw);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int i = tid + j * NT;
      const int zz = i / N, y = i - zz * N;
      if (par == 0)
        acc[j] = plane[zz * PITCH + y];
      else
        stv<T>(Sv, soff + i, acc[j] + mulc(plane[zz * PITCH + y], tw[y]));
    }
    __syncthreads();
  }
}

// =============================================================================================
// Class-split (y,z) pass.  The ky frequencies of the zero-padded 2n-point y-DFT are split into C
// classes ky = c (mod C).  For one class the DFT reduces to an M-point DFT (M = 2n / C) of the row
// folded onto M points with the twiddle exp(-i pi c y / n):
//     z_c[j] = sum_{m < n/M} x[j + m M] exp(-i pi c (j + m M) / n),
// and the cropped inverse of that class is the M-point inverse DFT Y_c, periodic in y with
// period M, times exp(+i pi c y / n).  One workgroup per (slot, kx, c) holds an n x M slab in LDS:
// fold, forward row DFTs, z-convolution of its M columns, inverse row DFTs, and writes Y_c to the
// class-major spectrum [c][kx][z][j] (or [c][z][kx][j], ClassCfg::ZMAJOR); k_xinv sums the
// classes.  C = 2 is the parity split of k_yz3 (no fold).  Larger C keeps the slab small enough
// for several workgroups per CU, so the global-memory phases of one workgroup overlap the
// transforms of another, and it lets grids whose whole n x n plane exceeds LDS (n = 192, 256) run
// the same way.
// Fold of one chunk for four classes (M = n / 2, two points per folded value) and class RC.
template <typename T, int N, int CH, int NT, int PITCH, int RC>
__device__ __forceinline__ void fold4(cplx<T>* slab, const cplx<T> (&xv)[CH][2], const cplx<T>* tw, int tid, int k0) {
  constexpr int M = N / 2;
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int idx = tid + (k0 + k) * NT;
    const int zz = idx / M, j = idx - zz * M;
    const cplx<T> x0 = xv[k][0], x1 = xv[k][1];
    cplx<T> acc = RC == 0 ? x0 + x1 : (RC == 1 ? x0 + mul_i<-1>(x1) : (RC == 2 ? x0 - x1 : x0 + mul_i<+1>(x1)));
    if constexpr (RC != 0) acc = acc * tw[(RC * j) % (2 * N)];
    slab[zz * PITCH + j] = acc;
  }
}

// Fold of one chunk for any class count: sum_m x_m exp(-i pi c (j + m M) / n).
template <typename T, int N, int M, int F, int CH, int NT, int PITCH>
__device__ __forceinline__ void foldg(cplx<T>* slab, const cplx<T> (&xv)[CH][F], const cplx<T>* tw, int tid, int k0,
                                      int c) {
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int idx = tid + (k0 + k) * NT;
    const int zz = idx / M, j = idx - zz * M;
    cplx<T> acc = c == 0 ? xv[k][0] : xv[k][0] * tw[(c * j) % (2 * N)];
#pragma unroll
    for (int m = 1; m < F; ++m) acc = acc + xv[k][m] * tw[(c * (j + m * M)) % (2 * N)];
    slab[zz * PITCH + j] = acc;
  }
}

template <typename T, int N>
struct ClassCfg {
  // number of classes; 2 = k_yz3 (complex64 at 64 and 96: four classes, fused, take the plane pass
  // from 0.294 to 0.243 and from 2.14 to 1.67 ms per 60-slot launch against the whole plane, for
  // 0.013 and 0.06 ms more in the x-inverse's class sum; six classes at 96: 1.99 ms, 0.13 ms more)
  static constexpr int C = N == 144 ? (sizeof(T) == 4 ? 6 : 18)
                          : sizeof(T) == 4 ? (N <= 32 ? 2 : (N <= 128 ? 4 : (N == 192 ? 6 : 8)))
                                           : (N <= 64 ? 2 : (N == 96 ? 6 : (N == 128 ? 8 : (N == 192 ? 12 : 16))));
  static constexpr int M = 2 * N / C;
  // complex64 from 192 up: one 100-140 KB slab per CU, worked on by 8 waves (fewer classes make
  // the class sum of the x-inverse cheaper than the lost overlap of two workgroups costs)
  static constexpr int NT = (sizeof(T) == 4 && N >= 192) ? 512 : 256;
  // waves per SIMD the register allocation must leave room for (complex128 at 128: two workgroups
  // per CU at the price of a few spilled registers)
  static constexpr int WPE = ((sizeof(T) == 8 && N == 128) || (sizeof(T) == 4 && N == 144)) ? 2 : 1;
  // z-convolution by the register four-step transform (else the in-LDS Stockham one; complex128
  // at 96 and 144 keeps the latter, which needs fewer registers).  144 = 4 x 36 is split for the
  // z-convolution only; its row transforms elsewhere stay Stockham.
  static constexpr bool ZFOUR = (HasSplit<N>::value || N == 144) && !(sizeof(T) == 8 && (N == 96 || N == 144));
  static constexpr int PITCH = M + 1;
  // fold and forward row DFTs straight from global memory, inverse row DFTs straight to it, with
  // R rows per lane group (complex64 at 64, 96, 128 and 192: 2.46 against 3.01 ms per 60-slot
  // launch at 128, 1.67 against 1.95 at 96); the other sizes stage both through the slab (measured
  // faster at 144 and 256, whose folds read three or four points per value; complex128 needs the
  // registers for its longer folds)
  static constexpr bool FUSED = sizeof(T) == 4 && (N == 64 || N == 96 || N == 128 || N == 192);
  // class output [c][z][kx][j] (else [c][kx][z][j]): the layout k_xinv's DFT class sum reads
  static constexpr bool ZMAJOR = XInvCfg<T, N>::dftsum(C);
  static_assert(C == 2 || (HasSplit<M>::value && N % M == 0 && M % 16 == 0), "class slab shape");
};

// twl[k1 * L + l] = exp(-2 pi i l k1 / M) from the 2n-entry table (stride 2n / M)
template <typename T, int M, int TWS>
__device__ __forceinline__ void fill_twl_stride(cplx<T>* twl, const cplx<T>* tw, int tid, int nt) {
  constexpr int L = Split<M>::L, E = Split<M>::E;
  for (int i = tid; i < L * E; i += nt) {
    const int k1 = i / L, l = i - k1 * L;
    twl[i] = tw[TWS * l * k1];
  }
}

// Folded values of R rows (lane holds j = lane + L e of row zz[r]), read straight from the plane:
// sum_m x[zz, j + m M] exp(-i pi c (j + m M) / n).  RC >= 0: four classes with two points per folded
// value, class RC (rho = exp(-2 pi i RC / 4) is a power of -i, so x_0 + rho x_1 is a register
// permutation, then one twiddle); RC < 0: any C.
template <typename T, int N, int M, int F, int R, int RC>
__device__ __forceinline__ void fold_rows(cplx<T> (&v)[R][Split<M>::E], const char* plane0, const int (&zz)[R],
                                          const cplx<T>* tw, int c, int lane) {
  constexpr int LM = Split<M>::L, EM = Split<M>::E;
  auto x = [&](int r, int e, int m) {
    return ldo<T>(plane0, (uint32_t)(zz[r] * N + lane + LM * e + m * M) * (uint32_t)sizeof(cplx<T>));
  };
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int e = 0; e < EM; ++e) {
      const int j = lane + LM * e;
      cplx<T> acc;
      if constexpr (RC >= 0) {
        const cplx<T> x0 = x(r, e, 0), x1 = x(r, e, 1);
        acc = RC == 0 ? x0 + x1 : (RC == 1 ? x0 + mul_i<-1>(x1) : (RC == 2 ? x0 - x1 : x0 + mul_i<+1>(x1)));
        if constexpr (RC != 0) acc = acc * tw[(RC * j) % (2 * N)];
      } else {
        acc = c == 0 ? x(r, e, 0) : x(r, e, 0) * tw[(c * j) % (2 * N)];
#pragma unroll
        for (int m = 1; m < F; ++m) acc = acc + x(r, e, m) * tw[(c * (j + m * M)) % (2 * N)];
      }
      v[r][e] = acc;
    }
}

// Rows handled together by one lane group in the row phases of k_yzc (1 when the groups do not
// divide the rows evenly, and in complex128, whose registers are taken by the z-convolution).
template <typename T, int N>
constexpr int yzc_rows() {
  constexpr int M = ClassCfg<T, N>::M, G = ClassCfg<T, N>::NT / Split<M>::L;
  return (N % G || sizeof(T) == 8) ? 1 : largest_divisor_upto(N / G, 2);
}

// Phase 1 of k_yzc for class value RC (or any class, RC < 0): fold, forward row DFT, spectrum to LDS.
template <typename T, int N, int RC>
__device__ __forceinline__ void yzc_rows_forward(cplx<T>* slab, const char* plane0, const cplx<T>* tw,
                                                 const cplx<T>* twlM, int c, int tid) {
  using CC = ClassCfg<T, N>;
  constexpr int M = CC::M, F = N / M, PITCH = CC::PITCH;
  constexpr int LM = Split<M>::L, EM = Split<M>::E, G = CC::NT / LM, R = yzc_rows<T, N>();
  const int g = tid / LM, lane = tid - g * LM;
#pragma unroll 1
  for (int idx0 = g; idx0 < N; idx0 += G * R) {
    cplx<T> v[R][EM];
    int zz[R];
#pragma unroll
    for (int r = 0; r < R; ++r) zz[r] = spreadL<N, LM>(idx0 + G * r);
    fold_rows<T, N, M, F, R, RC>(v, plane0, zz, tw, c, lane);
    cplx<T>* rows[R];
#pragma unroll
    for (int r = 0; r < R; ++r) rows[r] = slab + spreadL<N, LM>(idx0 + G * r) * PITCH;
    rows_a2b<T, M, -1, R>(v, rows, lane, twlM);
  }
}

template <typename T, int N>
__global__ __launch_bounds__((ClassCfg<T, N>::NT), (ClassCfg<T, N>::WPE)) void k_yzc(PassArgs a) {
  using CC = ClassCfg<T, N>;
  constexpr int C = CC::C, M = CC::M, NT = CC::NT, PITCH = CC::PITCH;
  constexpr int LM = Split<M>::L, EM = Split<M>::E;
  __shared__ cplx<T> slab[N * PITCH];
  __shared__ cplx<T> tw[2 * N];
  __shared__ cplx<T> twlM[M];
  __shared__ cplx<T> twlN[CC::ZFOUR ? N : 1];
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  // consecutive blocks on one XCD: the C classes of one (kx, slot) plane (the plane is read once
  // from HBM, then from L2), all slots of one kx (the kernel plane stays in L2), and kx in the
  // order 0, 1, 2n-1, 2, 2n-2, ..., n-1, n+1, n, so that kx and 2n - kx, which share a kernel
  // plane, follow each other (256^3: 0.46 GB less read per launch)
  const int lin = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int c = lin % C;
  const int ks = lin / C;
  const int sx = ks / a.nslots;
  const int slot = ks - sx * a.nslots;
  const int kx = sx == 0 ? 0 : (sx == 2 * N - 1 ? N : ((sx & 1) ? (sx + 1) / 2 : 2 * N - sx / 2));
  if (!slot_active(a, slot)) return;
  const int tid = threadIdx.x;
  const SlotDesc& d = a.desc[slot];
  const void* Sv = d.vec[a.spec];
  const size_t soff = (size_t)kx * N * N;
  const int kxp = kx <= N ? kx : 2 * N - kx;
  const cplx<T>* K = (const cplx<T>*)a.kern + (size_t)kxp * (4 * N * N);
  if constexpr (CC::FUSED) {
    for (int i = tid; i < 2 * N; i += NT) tw[i] = ld<T>(a.tw, i);
    __syncthreads();
    fill_twl_stride<T, M, C>(twlM, tw, tid, NT);
    if constexpr (CC::ZFOUR) fill_twl<T, N>(twlN, tw, tid, NT);
    __syncthreads();
    // phase 1: each lane group folds its rows straight from global memory into registers (the
    // y-DFT of the class is an M-point DFT of the folded row), transforms them and leaves the
    // spectra in LDS
    const char* plane0 = (const char*)Sv + soff * sizeof(cplx<T>);
    if constexpr (C == 4 && N / M == 2) {
      // class value uniform over the block: one specialised loop per value
      if (c == 0)
        yzc_rows_forward<T, N, 0>(slab, plane0, tw, twlM, c, tid);
      else if (c == 1)
        yzc_rows_forward<T, N, 1>(slab, plane0, tw, twlM, c, tid);
      else if (c == 2)
        yzc_rows_forward<T, N, 2>(slab, plane0, tw, twlM, c, tid);
      else
        yzc_rows_forward<T, N, 3>(slab, plane0, tw, twlM, c, tid);
    } else {
      yzc_rows_forward<T, N, -1>(slab, plane0, tw, twlM, c, tid);
    }
  } else {
    // fold through the slab, with the loads of a chunk issued together, then the row DFTs in LDS
    const char* plane0 = (const char*)Sv + soff * sizeof(cplx<T>);
    constexpr int F = N / M;
    constexpr int PER = N * M / NT;
    constexpr int CH0 = 32 / F < 8 ? 32 / F : 8;  // at most 32 loads in flight per thread
    constexpr int CH = largest_divisor_upto(PER, CH0);
    static_assert(PER % CH == 0 && PER * NT == N * M, "fold chunks");
    for (int i = tid; i < 2 * N; i += NT) tw[i] = ld<T>(a.tw, i);
#pragma unroll 1
    for (int k0 = 0; k0 < PER; k0 += CH) {
      cplx<T> xv[CH][F];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int idx = tid + (k0 + k) * NT;
        const int zz = idx / M, j = idx - zz * M;
#pragma unroll
        for (int m = 0; m < F; ++m)
          xv[k][m] = ldo<T>(plane0, (uint32_t)(zz * N + j + m * M) * (uint32_t)sizeof(cplx<T>));
      }
      if (k0 == 0) __syncthreads();  // tw visible
      foldg<T, N, M, F, CH, NT, PITCH>(slab, xv, tw, tid, k0, c);
    }
    fill_twl_stride<T, M, C>(twlM, tw, tid, NT);
    if constexpr (CC::ZFOUR) fill_twl<T, N>(twlN, tw, tid, NT);
    __syncthreads();
    constexpr int G = NT / LM;
    const int g = tid / LM, lane = tid - g * LM;
    for (int idx = g; idx < N; idx += G) row_fft<T, M, -1>(slab + spreadL<N, LM>(idx) * PITCH, lane, tw, twlM);
  }
  __syncthreads();
  // phase 2: z-convolution of the M columns of the slab
  if constexpr (CC::ZFOUR) {
    constexpr int L = Split<N>::L;
    constexpr int G = NT / L;
    const int g = tid / L, lane = tid - g * L;
    for (int idx = g; idx < M; idx += G) {
      const int j = spreadL<M, L>(idx);
      const int ky = c + C * spec_freq<M>(j);
      zconv4<T, N, PITCH>(slab + j, lane, tw, twlN, K + (size_t)ky * (2 * N));
    }
  } else {
    constexpr int L = Lanes<N>::value;
    constexpr int G = NT / L;
    const int g = tid / L, lane = tid - g * L;
    for (int idx = g; idx < M; idx += G) {
      const int j = spreadL<M, L>(idx);
      const int ky = c + C * spec_freq<M>(j);
      zconv<T, N>(slab + j, PITCH, lane, tw, K + (size_t)ky * (2 * N));
    }
  }
  __syncthreads();
  if constexpr (!CC::FUSED) {
    constexpr int G = NT / LM;
    const int g = tid / LM, lane = tid - g * LM;
    for (int idx = g; idx < N; idx += G) row_fft<T, M, +1>(slab + spreadL<N, LM>(idx) * PITCH, lane, tw, twlM);
    __syncthreads();
    void* Ov = d.vec[V_SPE];
    if constexpr (CC::ZMAJOR) {
      const size_t ooff = (size_t)c * 2 * N * N * M + (size_t)kx * M;
      for (int i = tid; i < N * M; i += NT) {
        const int zz = i / M, j = i - zz * M;
        stv<T>(Ov, ooff + (size_t)zz * (2 * N * M) + j, slab[zz * PITCH + j]);
      }
    } else {
      const size_t ooff = ((size_t)c * 2 * N + kx) * N * M;
      for (int i = tid; i < N * M; i += NT) {
        const int zz = i / M, j = i - zz * M;
        stv<T>(Ov, ooff + i, slab[zz * PITCH + j]);
      }
    }
  } else {
    // phase 3: inverse row DFTs from LDS into registers, written straight to the class-major output
    static_assert(!CC::ZMAJOR, "fused store writes [c][kx][z][j]");
    void* Ov = d.vec[V_SPE];
    const size_t ooff = ((size_t)c * 2 * N + kx) * N * M;
    constexpr int G = NT / LM, R = yzc_rows<T, N>();
    const int g = tid / LM, lane = tid - g * LM;
#pragma unroll 1
    for (int idx0 = g; idx0 < N; idx0 += G * R) {
      cplx<T> v[R][EM];
      cplx<T>* rows[R];
#pragma unroll
      for (int r = 0; r < R; ++r) rows[r] = slab + spreadL<N, LM>(idx0 + G * r) * PITCH;
      rows_b2a<T, M, +1, R>(v, rows, lane, twlM);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int zz = spreadL<N, LM>(idx0 + G * r);
#pragma unroll
        for (int e = 0; e < EM; ++e) stv<T>(Ov, ooff + (size_t)zz * M + lane + LM * e, v[r][e]);
      }
    }
  }
}

// Far field from n = 64 up: the z-rows of a kx plane are streamed through LDS in chunks, so no
// full plane is held and several workgroups share a CU.  Each thread owns one ky of the 2n-point accumulator.
template <typename T, int N>
__global__ __launch_bounds__(512) void k_ff_big(PassArgs a) {
  constexpr int R = 16, PITCH = N + 1, NT = 512;
  constexpr int L = row_lanes<N>();
  constexpr int NG = NT / L;
  __shared__ cplx<T> rE[R * PITCH];
  __shared__ cplx<T> rO[R * PITCH];
  __shared__ cplx<T> tw[2 * N];
  __shared__ cplx<T> twl[twl_size<N>()];
  int kx, slot;
  plane_decode(a, kx, slot);
  if (!slot_active(a, slot)) return;
  const int tid = threadIdx.x;
  const SlotDesc& d = a.desc[slot];
  for (int i = tid; i < 2 * N; i += NT) tw[i] = ld<T>(a.tw, i);
  __syncthreads();
  fill_twl_any<T, N>(twl, tw, tid, NT);
  const void* Sv = d.vec[a.spec];
  const size_t soff = (size_t)kx * N * N;
  const int kxp = kx <= N ? kx : 2 * N - kx;
  const cplx<T>* K = (const cplx<T>*)a.kern + (size_t)kxp * (2 * N * N);
  const int g = tid / L, lane = tid - g * L;
  cplx<T> acc = {0, 0};
  for (int z0 = 0; z0 < N; z0 += R) {
    __syncthreads();
    for (int idx = tid; idx < R * N; idx += NT) {
      const int r = idx / N, y = idx - r * N;
      const cplx<T> v = ld<T>(Sv, soff + (size_t)(z0 + r) * N + y);
      rE[r * PITCH + y] = v;
      rO[r * PITCH + y] = v * tw[y];
    }
    __syncthreads();
    for (int u = g; u < 2 * R; u += NG) row_fft<T, N, -1>(u < R ? rE + u * PITCH : rO + (u - R) * PITCH, lane, tw, twl);
    __syncthreads();
    if (tid < 2 * N) {
      const int ky = tid;
      const cplx<T>* src = (ky & 1) ? rO : rE;
      const int pos = spec_pos<N>(ky >> 1);
      for (int r = 0; r < R; ++r) acc = acc + ld<T>(K, (size_t)(z0 + r) * 2 * N + ky) * src[r * PITCH + pos];
    }
  }
  __syncthreads();
  if (tid < 2 * N) ((tid & 1) ? rO : rE)[spec_pos<N>(tid >> 1)] = acc;
  __syncthreads();
  if (g < 2) row_fft<T, N, +1>(g == 0 ? rE : rO, lane, tw, twl);
  __syncthreads();
  void* out = d.vec[a.sel];
  for (int y = tid; y < N; y += NT) stv<T>(out, (size_t)kx * N + y, rE[y] + mulc(rO[y], tw[y]));
}

template <typename T, int N>
__global__ __launch_bounds__(512) void k_ffT_big(PassArgs a) {
  constexpr int R = 16, PITCH = N + 1, NT = 512;
  constexpr int L = row_lanes<N>();
  constexpr int NG = NT / L;
  __shared__ cplx<T> rE[R * PITCH];
  __shared__ cplx<T> rO[R * PITCH];
  __shared__ cplx<T> hat[2 * N];
  __shared__ cplx<T> tw[2 * N];
  __shared__ cplx<T> twl[twl_size<N>()];
  int kx, slot;
  plane_decode(a, kx, slot);
  if (!slot_active(a, slot)) return;
  const int tid = threadIdx.x;
  const SlotDesc& d = a.desc[slot];
  for (int i = tid; i < 2 * N; i += NT) tw[i] = ld<T>(a.tw, i);
  __syncthreads();
  fill_twl_any<T, N>(twl, tw, tid, NT);
  const void* rowv = d.vec[a.sel];
  for (int y = tid; y < N; y += NT) {
    const cplx<T> v = ld<T>(rowv, (size_t)kx * N + y);
    hat[y] = v;
    hat[N + y] = v * tw[y];
  }
  __syncthreads();
  const int g = tid / L, lane = tid - g * L;
  if (g < 2) row_fft<T, N, -1>(hat + g * N, lane, tw, twl);
  __syncthreads();
  void* Sv = d.vec[a.spec];
  const size_t soff = (size_t)kx * N * N;
  const int kxp = kx <= N ? kx : 2 * N - kx;
  const cplx<T>* K = (const cplx<T>*)a.kern + (size_t)kxp * (2 * N * N);
  for (int z0 = 0; z0 < N; z0 += R) {
    for (int idx = tid; idx < R * 2 * N; idx += NT) {
      const int r = idx / (2 * N), ky = idx - r * 2 * N;
      const int pos = spec_pos<N>(ky >> 1);
      const cplx<T> v = ld<T>(K, (size_t)(z0 + r) * 2 * N + ky) * hat[(ky & 1) * N + pos];
      ((ky & 1) ? rO : rE)[r * PITCH + pos] = v;
    }
    __syncthreads();
    for (int u = g; u < 2 * R; u += NG) row_fft<T, N, +1>(u < R ? rE + u * PITCH : rO + (u - R) * PITCH, lane, tw, twl);
    __syncthreads();
    for (int idx = tid; idx < R * N; idx += NT) {
      const int r = idx / N, y = idx - r * N;
      stv<T>(Sv, soff + (size_t)(z0 + r) * N + y, rE[r * PITCH + y] + mulc(rO[r * PITCH + y], tw[y]));
    }
    __syncthreads();
  }
}

// =============================================================================================
// BiCGSTAB vector update x += alpha p + omega s, r = s - omega t, with <rh, r> and ||r||^2.
template <typename T, int N>
__global__ __launch_bounds__(256) void k_update(PassArgs a) {
  using X = XCfg<N>;
  constexpr int TY = X::TY, NYT = X::NYT, IT = X::IT;
  __shared__ double red[4 * 4];
  const int tid = threadIdx.x;
  // XCD-aware slot-major order from n = 192 up (measured at 256^3: 9.42 against 9.83 ms; at 96,
  // 128 and 144 launch order is as fast or faster: complex64 at 128, 1.20 against 1.26 ms)
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int lin = (N >= 192 && nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int per = a.nz * NYT;
  const int slot = lin / per;
  const int blk = lin - slot * per;
  if (!slot_active(a, slot)) return;
  const SlotDesc& d = a.desc[slot];
  const SlotState& st = a.st[slot];
  const size_t row0 = (size_t)blk * TY * N;
  const cplx<T> alpha = scal<T>(st.alpha), omega = scal<T>(st.omega);
  if (st.status == ST_HALF) {
    for (int i = tid; i < TY * N; i += 256) {
      const size_t idx = row0 + i;
      stv<T>(d.vec[V_X], idx, ldn<T>(d.vec[V_X], idx) + alpha * ldn<T>(d.vec[V_P], idx));
    }
    return;
  }
  cplx<T> xs[IT], ps[IT], ss[IT], ts[IT], hs[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int i = tid + it * 256;
    if (i < TY * N) {
      const size_t idx = row0 + i;
      xs[it] = ldn<T>(d.vec[V_X], idx);
      ps[it] = ldn<T>(d.vec[V_P], idx);
      ss[it] = ldn<T>(d.vec[V_S], idx);
      ts[it] = ldn<T>(d.vec[V_T], idx);
      hs[it] = ldn<T>(d.vec[V_RH], idx);
    }
  }
  cplx<double> rho = {0, 0};
  double rr = 0.0;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int i = tid + it * 256;
    if (i < TY * N) {
      const size_t idx = row0 + i;
      stv<T>(d.vec[V_X], idx, xs[it] + alpha * ps[it] + omega * ss[it]);
      const cplx<T> r = ss[it] - omega * ts[it];
      stv<T>(d.vec[V_R], idx, r);
      dot_acc(rho, hs[it], r);
      rr += (double)r.re * r.re + (double)r.im * r.im;
    }
  }
  double v[3] = {rho.re, rho.im, rr};
  block_sum<3>(v, red);
  if (tid == 0) {
    double* pp = part_ptr(a, slot, blk, 0);
    pp[0] = v[0];
    pp[1] = v[1];
    pp[2] = v[2];
    pp[3] = 0.0;
  }
}

// =============================================================================================
// Per-slot scalar step of BiCGSTAB.  One block per slot sums the block partials in a fixed
// order (deterministic), then thread 0 advances the recurrence in FP64 complex arithmetic.
__device__ __forceinline__ cplx<double> cdiv(cplx<double> a, cplx<double> b) {
  const double den = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den};
}
__device__ __forceinline__ cplx<double> cmul(cplx<double> a, cplx<double> b) { return a * b; }
__device__ __forceinline__ cplx<double> getc(const double* v) { return {v[0], v[1]}; }
__device__ __forceinline__ void putc(double* v, cplx<double> c) {
  v[0] = c.re;
  v[1] = c.im;
}

__device__ __forceinline__ void fresh_restart(SlotState& st) {
  // rh = r (applied by the next p-update), p = v = 0, rho_prev = alpha = omega = 1
  st.restart_flag = 1;
  st.nrh = st.rr;
  st.rho[0] = st.rr * st.rr;
  st.rho[1] = 0.0;
  st.rho_prev[0] = st.alpha[0] = st.omega[0] = 1.0;
  st.rho_prev[1] = st.alpha[1] = st.omega[1] = 0.0;
}

__device__ __forceinline__ bool final_state(int s) {
  return s == ST_OK || s == ST_MAXIT || s == ST_BREAK || s == ST_NONFIN;
}

template <int KIND>
__device__ __forceinline__ void scalar_update(SlotState& st, const double (&v)[6]);

template <int KIND>
__global__ __launch_bounds__(256) void k_scalar(PassArgs a) {
  __shared__ double red[6 * 4];
  const int slot = blockIdx.x;
  if (!slot_active(a, slot)) return;
  const int tid = threadIdx.x;
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int b = tid; b < a.part_stride; b += 256) {
    const double* pp = a.part + ((size_t)slot * a.part_stride + b) * PART_K * 2;
#pragma unroll
    for (int j = 0; j < 6; ++j) v[j] += pp[j];
  }
  block_sum<6>(v, red);
  if (tid != 0) return;
  SlotState& st = a.st[slot];
  const int s0 = st.status;
  scalar_update<KIND>(st, v);
  if (final_state(st.status) && !final_state(s0)) st.t_done = (uint64_t)wall_clock64();
}

// One step of the per-slot BiCGSTAB scalar recurrence from the block-summed partials v.
template <int KIND>
__device__ __forceinline__ void scalar_update(SlotState& st, const double (&v)[6]) {
  const cplx<double> p0 = {v[0], v[1]}, p1 = {v[2], v[3]}, p2 = {v[4], v[5]};
  if (KIND == SC_INIT) {
    st.matvecs += 1;
    st.nb = sqrt(p1.re);
    st.rr = sqrt(p0.re);
    if (!(st.nb > 0.0)) {
      st.relres = st.relres_true = 0.0;
      st.status = isfinite(st.nb) ? ST_OK : ST_NONFIN;
      return;
    }
    st.relres = st.rr / st.nb;
    if (!isfinite(st.relres)) {
      st.status = ST_NONFIN;
      return;
    }
    if (st.relres <= st.tol) {
      st.relres_true = st.relres;
      st.status = ST_OK;
      return;
    }
    fresh_restart(st);
    st.restart_flag = 1;
    st.beta[0] = st.rho[0];
    st.beta[1] = 0.0;
    st.status = ST_RUN;
  } else if (KIND == SC_ALPHA) {
    st.matvecs += 1;
    const cplx<double> rv = p0;
    const cplx<double> al = cdiv(getc(st.rho), rv);
    if (!(isfinite(al.re) && isfinite(al.im))) {
      st.status = (rv.re == 0.0 && rv.im == 0.0) ? ST_BREAK : ST_NONFIN;
      return;
    }
    putc(st.alpha, al);
    st.restart_flag = 0;
  } else if (KIND == SC_OMEGA) {
    st.matvecs += 1;
    const double ns = sqrt(p0.re);
    if (ns / st.nb <= st.tol) {
      st.rr = ns;
      st.status = ST_HALF;
      return;
    }
    const cplx<double> om = {p1.re / p2.re, p1.im / p2.re};
    if (!(isfinite(om.re) && isfinite(om.im))) {
      st.status = ST_NONFIN;
      return;
    }
    putc(st.omega, om);
  } else if (KIND == SC_BETA) {
    st.iters += 1;
    if (st.status == ST_HALF) {
      st.relres = st.rr / st.nb;
      st.status = ST_CHECK;
      return;
    }
    st.rho_prev[0] = st.rho[0];
    st.rho_prev[1] = st.rho[1];
    st.rr = sqrt(v[2]);
    st.relres = st.rr / st.nb;
    if (!isfinite(st.relres)) {
      st.status = ST_NONFIN;
      return;
    }
    if (st.relres <= st.tol || st.iters >= st.maxit) {
      st.status = ST_CHECK;
      return;
    }
    cplx<double> rho = p0;
    const bool om_zero = st.omega[0] == 0.0 && st.omega[1] == 0.0;
    if (om_zero || sqrt(rho.re * rho.re + rho.im * rho.im) <= st.brk * st.nrh * st.rr) {
      st.restarts += 1;
      fresh_restart(st);
      rho = getc(st.rho);
    }
    const cplx<double> be = cmul(cdiv(rho, getc(st.rho_prev)), cdiv(getc(st.alpha), getc(st.omega)));
    putc(st.beta, be);
    putc(st.rho, rho);
  } else if (KIND == SC_FINAL) {
    st.matvecs += 1;
    const double rt = sqrt(p0.re);
    st.relres_true = rt / st.nb;
    if (st.relres_true <= st.tol) {
      st.status = ST_OK;
    } else if (st.iters >= st.maxit) {
      st.status = ST_MAXIT;
    } else if (st.restarts >= st.max_restarts) {
      st.status = ST_BREAK;
    } else {
      st.rr = rt;
      st.restarts += 1;
      fresh_restart(st);
      st.beta[0] = st.rho[0];
      st.beta[1] = 0.0;
      st.status = ST_RUN;
    }
  }
}

// =============================================================================================
// grad[i] (+)= sum_q w_q Re(u_q[i] wbar_q[i]), summed over slots in index order in FP64.
template <typename T>
__global__ __launch_bounds__(256) void k_grad_accum(const SlotDesc* desc, const double* w, int nslots, int sel_u,
                                                    int sel_w, double* grad, size_t N, int accumulate) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  double s = accumulate ? grad[i] : 0.0;
  for (int q = 0; q < nslots; ++q) {
    const cplx<T> u = ld<T>(desc[q].vec[sel_u], i);
    const cplx<T> wb = ld<T>(desc[q].vec[sel_w], i);
    const double wq = w ? 1.0 / w[2 * q + 1] : 1.0;
    s += wq * ((double)u.re * wb.re - (double)u.im * wb.im);
  }
  grad[i] = s;
}

// grad[i] (+)= sum_q w_q Re(u_q[i] wb_q[i]) over contiguous [Q][N] arrays, FP64 sum in q order.
template <typename T>
__global__ __launch_bounds__(256) void k_grad_sum(const cplx<T>* u, const cplx<T>* wb, int Q, size_t N,
                                                  const double* stats, T* grad, int accumulate) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  double s = accumulate ? (double)grad[i] : 0.0;
  for (int q = 0; q < Q; ++q) {
    const cplx<T> a = u[(size_t)q * N + i], b = wb[(size_t)q * N + i];
    const double wq = stats ? 1.0 / stats[2 * q + 1] : 1.0;
    s += wq * ((double)a.re * b.re - (double)a.im * b.im);
  }
  grad[i] = (T)s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_convert(const double* src, T* dst, size_t N) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < N) dst[i] = (T)src[i];
}

// r = w_q (y - ymeas) per view with FP64 ||y - ymeas||^2 and ||ymeas||^2 (one block per view, fixed
// order); w_q = 1, or 1 / ||ymeas_q||^2 when WEIGHTED (then ||ymeas||^2 is summed in a first sweep).
template <typename T, bool WEIGHTED>
__global__ __launch_bounds__(256) void k_residual(const cplx<T>* y, const cplx<T>* ym, int M, cplx<T>* r,
                                                  double* stats) {
  __shared__ double red[2 * 4];
  __shared__ double nym;
  const int q = blockIdx.x;
  double v[2] = {0, 0};
  T w = (T)1;
  if (WEIGHTED) {
    double s1[1] = {0.0};
    for (int i = threadIdx.x; i < M; i += 256) {
      const cplx<T> b = ym[(size_t)q * M + i];
      s1[0] += (double)b.re * b.re + (double)b.im * b.im;
    }
    block_sum<1>(s1, red);
    if (threadIdx.x == 0) nym = s1[0];
    __syncthreads();
    v[1] = nym;
    w = (T)(1.0 / v[1]);
  }
  for (int i = threadIdx.x; i < M; i += 256) {
    const size_t idx = (size_t)q * M + i;
    const cplx<T> a = y[idx], b = ym[idx];
    const cplx<T> d = a - b;
    r[idx] = WEIGHTED ? cplx<T>{d.re * w, d.im * w} : d;
    v[0] += (double)d.re * d.re + (double)d.im * d.im;
    if (!WEIGHTED) v[1] += (double)b.re * b.re + (double)b.im * b.im;
  }
  if (WEIGHTED) {
    double s0[1] = {v[0]};
    block_sum<1>(s0, red);
    v[0] = s0[0];
  } else {
    block_sum<2>(v, red);
  }
  if (threadIdx.x == 0) {
    stats[2 * q] = v[0];
    stats[2 * q + 1] = v[1];
  }
}

// Data term of eq. (prob) from the per-view sums: sum_q stats[2q] / (2 stats[2q+1]) in q order.
__global__ void k_data_loss(const double* stats, int Q, double* loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int q = 0; q < Q; ++q) s += stats[2 * q] / (2.0 * stats[2 * q + 1]);
  *loss = s;
}

// =============================================================================================
// launchers
template <typename T, int N>
static hipError_t xfwd_t(const PassArgs& a, hipStream_t s) {
  const dim3 nb(a.nslots * a.nz * XCfg<N>::NYT);
  switch (a.mode) {
    case PRO_F_VEC: hipLaunchKernelGGL((k_xfwd<T, N, PRO_F_VEC>), nb, dim3(256), 0, s, a); break;
    case PRO_F_B: hipLaunchKernelGGL((k_xfwd<T, N, PRO_F_B>), nb, dim3(256), 0, s, a); break;
    case PRO_P: hipLaunchKernelGGL((k_xfwd<T, N, PRO_P>), nb, dim3(256), 0, s, a); break;
    case PRO_S: hipLaunchKernelGGL((k_xfwd<T, N, PRO_S>), nb, dim3(256), 0, s, a); break;
    case PRO_VEC: hipLaunchKernelGGL((k_xfwd<T, N, PRO_VEC>), nb, dim3(256), 0, s, a); break;
    case PRO_CONJ_VEC: hipLaunchKernelGGL((k_xfwd<T, N, PRO_CONJ_VEC>), nb, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template <typename T, int N>
static hipError_t xinv_t(const PassArgs& a, hipStream_t s) {
  const dim3 nb(a.nslots * a.nz * XCfg<N>::NYT);
  constexpr int CL = ClassCfg<T, N>::C;
  if (a.spec2 < 0) {  // plain spectrum (far-field transpose)
    if (a.mode != EPI_STORE) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_xinv<T, N, EPI_STORE, 1>), nb, dim3(XInvCfg<T, N>::NT), 0, s, a);
    return hipGetLastError();
  }
  // the class output of the (y,z) pass covers whole volumes (its layout assumes n z-rows)
  if (a.nz != N) return hipErrorInvalidValue;
  switch (a.mode) {
    case EPI_STORE: hipLaunchKernelGGL((k_xinv<T, N, EPI_STORE, CL>), nb, dim3(XInvCfg<T, N>::NT), 0, s, a); break;
    case EPI_AXV: hipLaunchKernelGGL((k_xinv<T, N, EPI_AXV, CL>), nb, dim3(XInvCfg<T, N>::NT), 0, s, a); break;
    case EPI_AXT: hipLaunchKernelGGL((k_xinv<T, N, EPI_AXT, CL>), nb, dim3(XInvCfg<T, N>::NT), 0, s, a); break;
    case EPI_R0: hipLaunchKernelGGL((k_xinv<T, N, EPI_R0, CL>), nb, dim3(XInvCfg<T, N>::NT), 0, s, a); break;
    case EPI_TRUE: hipLaunchKernelGGL((k_xinv<T, N, EPI_TRUE, CL>), nb, dim3(XInvCfg<T, N>::NT), 0, s, a); break;
    case EPI_R0X: hipLaunchKernelGGL((k_xinv<T, N, EPI_R0X, CL>), nb, dim3(XInvCfg<T, N>::NT), 0, s, a); break;
    case EPI_AX: hipLaunchKernelGGL((k_xinv<T, N, EPI_AX, CL>), nb, dim3(XInvCfg<T, N>::NT), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template <typename T, int N>
static hipError_t update_t(const PassArgs& a, hipStream_t s) {
  const int nb = a.nslots * a.nz * (N / (N < 16 ? N : 16));
  hipLaunchKernelGGL((k_update<T, N>), dim3(nb), dim3(256), 0, s, a);
  return hipGetLastError();
}
// Far field and its transpose: from n = 64 up the kernels that stream 16 z-rows at a time
// through LDS are used (measured 1.3-1.4x faster at n = 64..128 than holding the whole plane,
// which allows one workgroup per CU); the whole-plane kernels serve the small grids.
template <typename T, int N>
constexpr bool split_plane() {
  return N > 32;
}
template <typename T, int N>
static hipError_t yz_t(const PassArgs& a, hipStream_t s) {
  using CC = ClassCfg<T, N>;
  if constexpr (CC::C == 2)
    hipLaunchKernelGGL((k_yz3<T, N>), dim3(a.nslots * 2 * N * 2), dim3(Plane3Cfg<N>::NT), 0, s, a);
  else
    hipLaunchKernelGGL((k_yzc<T, N>), dim3(a.nslots * 2 * N * CC::C), dim3(CC::NT), 0, s, a);
  return hipGetLastError();
}
template <typename T, int N>
static hipError_t ff_t(const PassArgs& a, hipStream_t s) {
  if constexpr (split_plane<T, N>())
    hipLaunchKernelGGL((k_ff_big<T, N>), dim3(a.nslots * 2 * N), dim3(512), 0, s, a);
  else
    hipLaunchKernelGGL((k_ff<T, N>), dim3(a.nslots * 2 * N), dim3(PlaneCfg<N>::NT), 0, s, a);
  return hipGetLastError();
}
template <typename T, int N>
static hipError_t ffT_t(const PassArgs& a, hipStream_t s) {
  if constexpr (split_plane<T, N>())
    hipLaunchKernelGGL((k_ffT_big<T, N>), dim3(a.nslots * 2 * N), dim3(512), 0, s, a);
  else
    hipLaunchKernelGGL((k_ffT<T, N>), dim3(a.nslots * 2 * N), dim3(PlaneCfg<N>::NT), 0, s, a);
  return hipGetLastError();
}

#define LS_DISPATCH_F(FN, n, ...)                         \
  switch (n) {                                            \
    case 8: return FN<float, 8>(__VA_ARGS__);             \
    case 16: return FN<float, 16>(__VA_ARGS__);           \
    case 32: return FN<float, 32>(__VA_ARGS__);           \
    case 64: return FN<float, 64>(__VA_ARGS__);           \
    case 96: return FN<float, 96>(__VA_ARGS__);           \
    case 128: return FN<float, 128>(__VA_ARGS__);         \
    case 144: return FN<float, 144>(__VA_ARGS__);         \
    case 192: return FN<float, 192>(__VA_ARGS__);         \
    case 256: return FN<float, 256>(__VA_ARGS__);         \
    default: return hipErrorInvalidValue;                 \
  }
#define LS_DISPATCH_D(FN, n, ...)                         \
  switch (n) {                                            \
    case 8: return FN<double, 8>(__VA_ARGS__);            \
    case 16: return FN<double, 16>(__VA_ARGS__);          \
    case 32: return FN<double, 32>(__VA_ARGS__);          \
    case 64: return FN<double, 64>(__VA_ARGS__);          \
    case 96: return FN<double, 96>(__VA_ARGS__);          \
    case 128: return FN<double, 128>(__VA_ARGS__);        \
    case 144: return FN<double, 144>(__VA_ARGS__);        \
    case 192: return FN<double, 192>(__VA_ARGS__);        \
    case 256: return FN<double, 256>(__VA_ARGS__);        \
    default: return hipErrorInvalidValue;                 \
  }
#define LS_DISPATCH(FN, dbl, n, ...)   \
  if (dbl) {                           \
    LS_DISPATCH_D(FN, n, __VA_ARGS__)  \
  } else {                             \
    LS_DISPATCH_F(FN, n, __VA_ARGS__)  \
  }

bool fused_supported(int n, bool dbl) {
  (void)dbl;
  return n == 8 || n == 16 || n == 32 || n == 64 || n == 96 || n == 128 || n == 144 || n == 192 || n == 256;
}


hipError_t launch_xfwd(bool dbl, int n, const PassArgs& a, hipStream_t s) { LS_DISPATCH(xfwd_t, dbl, n, a, s) }
hipError_t launch_xinv(bool dbl, int n, const PassArgs& a, hipStream_t s) { LS_DISPATCH(xinv_t, dbl, n, a, s) }
hipError_t launch_yz(bool dbl, int n, const PassArgs& a, hipStream_t s) { LS_DISPATCH(yz_t, dbl, n, a, s) }
hipError_t launch_ff(bool dbl, int n, const PassArgs& a, hipStream_t s) { LS_DISPATCH(ff_t, dbl, n, a, s) }
hipError_t launch_ffT(bool dbl, int n, const PassArgs& a, hipStream_t s) { LS_DISPATCH(ffT_t, dbl, n, a, s) }
hipError_t launch_update(bool dbl, int n, const PassArgs& a, hipStream_t s) { LS_DISPATCH(update_t, dbl, n, a, s) }

hipError_t launch_scalar(int kind, bool dbl, const PassArgs& a, hipStream_t s) {
  (void)dbl;
  switch (kind) {
    case SC_INIT: hipLaunchKernelGGL(k_scalar<SC_INIT>, dim3(a.nslots), dim3(256), 0, s, a); break;
    case SC_ALPHA: hipLaunchKernelGGL(k_scalar<SC_ALPHA>, dim3(a.nslots), dim3(256), 0, s, a); break;
    case SC_OMEGA: hipLaunchKernelGGL(k_scalar<SC_OMEGA>, dim3(a.nslots), dim3(256), 0, s, a); break;
    case SC_BETA: hipLaunchKernelGGL(k_scalar<SC_BETA>, dim3(a.nslots), dim3(256), 0, s, a); break;
    case SC_FINAL: hipLaunchKernelGGL(k_scalar<SC_FINAL>, dim3(a.nslots), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_grad_accum(bool dbl, int n, const SlotDesc* desc, const double* w, int nslots, int sel_u,
                             int sel_w, void* grad, int accumulate, hipStream_t s) {
  const size_t N = (size_t)n * n * n;
  const int nb = (int)((N + 255) / 256);
  if (dbl)
    hipLaunchKernelGGL(k_grad_accum<double>, dim3(nb), dim3(256), 0, s, desc, w, nslots, sel_u, sel_w, (double*)grad,
                       N, accumulate);
  else
    hipLaunchKernelGGL(k_grad_accum<float>, dim3(nb), dim3(256), 0, s, desc, w, nslots, sel_u, sel_w, (double*)grad,
                       N, accumulate);
  return hipGetLastError();
}

hipError_t launch_grad_sum(bool dbl, const void* u, const void* wb, int Q, size_t N, const double* stats, void* grad,
                           int accumulate, hipStream_t s) {
  const int nb = (int)((N + 255) / 256);
  if (dbl)
    hipLaunchKernelGGL(k_grad_sum<double>, dim3(nb), dim3(256), 0, s, (const cplx<double>*)u,
                       (const cplx<double>*)wb, Q, N, stats, (double*)grad, accumulate);
  else
    hipLaunchKernelGGL(k_grad_sum<float>, dim3(nb), dim3(256), 0, s, (const cplx<float>*)u, (const cplx<float>*)wb,
                       Q, N, stats, (float*)grad, accumulate);
  return hipGetLastError();
}

hipError_t launch_convert(bool dbl, const double* src, void* dst, size_t N, hipStream_t s) {
  const int nb = (int)((N + 255) / 256);
  if (dbl)
    hipLaunchKernelGGL(k_convert<double>, dim3(nb), dim3(256), 0, s, src, (double*)dst, N);
  else
    hipLaunchKernelGGL(k_convert<float>, dim3(nb), dim3(256), 0, s, src, (float*)dst, N);
  return hipGetLastError();
}

hipError_t launch_residual(bool dbl, int m, const void* y, const void* ymeas, int Q, bool weighted, void* r,
                           double* stats, double* loss, hipStream_t s) {
  const int M = m * m;
  if (dbl) {
    if (weighted)
      hipLaunchKernelGGL((k_residual<double, true>), dim3(Q), dim3(256), 0, s, (const cplx<double>*)y,
                         (const cplx<double>*)ymeas, M, (cplx<double>*)r, stats);
    else
      hipLaunchKernelGGL((k_residual<double, false>), dim3(Q), dim3(256), 0, s, (const cplx<double>*)y,
                         (const cplx<double>*)ymeas, M, (cplx<double>*)r, stats);
  } else {
    if (weighted)
      hipLaunchKernelGGL((k_residual<float, true>), dim3(Q), dim3(256), 0, s, (const cplx<float>*)y,
                         (const cplx<float>*)ymeas, M, (cplx<float>*)r, stats);
    else
      hipLaunchKernelGGL((k_residual<float, false>), dim3(Q), dim3(256), 0, s, (const cplx<float>*)y,
                         (const cplx<float>*)ymeas, M, (cplx<float>*)r, stats);
  }
  if (loss) hipLaunchKernelGGL(k_data_loss, dim3(1), dim3(64), 0, s, stats, Q, loss);
  return hipGetLastError();
}

}  // namespace ls
