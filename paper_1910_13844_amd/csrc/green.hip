// Construction of the Fourier-domain Green kernels (run once per geometry, FP64 throughout).
//
// Volume kernel (Proposition 2): for every s in [[0, p/2-1]]^3 the samples
// ghat_t(delta |(p/2) q' - s|), q' in Omega_{2n}, are inverse-transformed on the 2n grid and
// accumulated with the phase exp(-2 i pi k.s / (n p)) (k the signed index in Omega_{2n});
// one forward 3D DFT of the sum gives ghat_m.  Only the 2n grid is ever allocated.
//
// Far-field kernels (Section on G~): for every z-slice, the free-space Green function
// g(dx, dy, x_Gamma - z) sampled at lateral offsets in Omega_{2n}^2 and 2D-transformed.
#include "fft.hpp"
#include "green.hpp"

#include <cmath>
#include <vector>

namespace ls {

__device__ __forceinline__ int sgn_index(int j, int M) { return j <= M / 2 ? j : j - M; }

// Transform of the Green function truncated at radius R, at radial frequency s >= 0.
// With E(a) = int_0^R e^{i a r} dr = R e^{i a R/2} sinc(a R/2):
//   ghat_t(s) = (E(k+s) - E(k-s)) / (2 i s),   ghat_t(0) = (e^{ikR}(1 - ikR) - 1)/k^2.
// This equals eq. (GreenL) with the sinc term's sign taken as minus (the reading under which
// eq. (GreenL2) is its continuous extension), without its removable singularity at s = k.
__device__ cplx<double> ghat_trunc(double s, double k, double R) {
  if (s == 0.0) {
    const double c = cos(k * R), sn = sin(k * R);
    return {(c + k * R * sn - 1.0) / (k * k), (sn - k * R * c) / (k * k)};
  }
  double e1r, e1i, e2r, e2i;
  {
    const double x = 0.5 * (k + s) * R;
    const double sc = x == 0.0 ? 1.0 : sin(x) / x;
    e1r = R * sc * cos(x);
    e1i = R * sc * sin(x);
  }
  {
    const double x = 0.5 * (k - s) * R;
    const double sc = x == 0.0 ? 1.0 : sin(x) / x;
    e2r = R * sc * cos(x);
    e2i = R * sc * sin(x);
  }
  const double nr = e1r - e2r, ni = e1i - e2i;
  return {ni / (2.0 * s), -nr / (2.0 * s)};
}

__global__ void k_fill_ghat(cplx<double>* B, int n, int half, int s0, int s1, int s2, double k, double R,
                            double delta) {
  const int M = 2 * n;
  const size_t tot = (size_t)M * M * M;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot; idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / ((size_t)M * M));
    const int j = (int)((idx / M) % M);
    const int l = (int)(idx % M);
    const double a = (double)(half * sgn_index(i, M) - s0);
    const double b = (double)(half * sgn_index(j, M) - s1);
    const double c = (double)(half * sgn_index(l, M) - s2);
    B[idx] = ghat_trunc(delta * sqrt(a * a + b * b + c * c), k, R);
  }
}

__global__ void k_accum_phase(cplx<double>* acc, const cplx<double>* B, int n, int p, int s0, int s1, int s2,
                              int first) {
  const int M = 2 * n;
  const size_t tot = (size_t)M * M * M;
  const double two_pi_over = 2.0 * M_PI / ((double)n * p);
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot; idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / ((size_t)M * M));
    const int j = (int)((idx / M) % M);
    const int l = (int)(idx % M);
    const double ph = -two_pi_over * ((double)sgn_index(i, M) * s0 + (double)sgn_index(j, M) * s1 +
                                      (double)sgn_index(l, M) * s2);
    double sn, cs;
    sincos(ph, &sn, &cs);
    const cplx<double> v = B[idx] * cplx<double>{cs, sn};
    acc[idx] = first ? v : acc[idx] + v;
  }
}

// g(|(dx, dy, Z)|) on the 2n-periodic lateral offset grid, one plane per slice z.
__global__ void k_fill_ffslices(cplx<double>* B, int n, double k, double xg) {
  const int M = 2 * n;
  const size_t tot = (size_t)n * M * M;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot; idx += (size_t)gridDim.x * blockDim.x) {
    const int z = (int)(idx / ((size_t)M * M));
    const int a = (int)((idx / M) % M);
    const int b = (int)(idx % M);
    const double Z = xg - (double)(z - n / 2 + 1);
    const double dy = (double)sgn_index(a, M), dx = (double)sgn_index(b, M);
    const double r = sqrt(dx * dx + dy * dy + Z * Z);
    double sn, cs;
    sincos(k * r, &sn, &cs);
    const double w = 1.0 / (4.0 * M_PI * r);
    B[idx] = {w * cs, w * sn};
  }
}

template <typename T>
__global__ void k_pack_vol(cplx<T>* K, const cplx<double>* G, int n, double scale) {
  const int M = 2 * n;
  const size_t tot = (size_t)(n + 1) * M * M;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot; idx += (size_t)gridDim.x * blockDim.x) {
    const cplx<double> v = G[idx];
    K[idx] = cplx<T>{(T)(v.re * scale), (T)(v.im * scale)};
  }
}

// Kff[kx'][z][ky] = F[z][ky][kx'] * scale, kx' in [0, n]
template <typename T>
__global__ void k_pack_ff(cplx<T>* K, const cplx<double>* F, int n, double scale) {
  const int M = 2 * n;
  const size_t tot = (size_t)(n + 1) * n * M;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot; idx += (size_t)gridDim.x * blockDim.x) {
    const int kxp = (int)(idx / ((size_t)n * M));
    const int z = (int)((idx / M) % n);
    const int ky = (int)(idx % M);
    const cplx<double> v = F[((size_t)z * M + ky) * M + kxp];
    K[idx] = cplx<T>{(T)(v.re * scale), (T)(v.im * scale)};
  }
}

// ---------------------------------------------------------------------------------------------
// FP64 full-length FFTs along one axis of a batch of lines.
// Contiguous lines: block handles 256/L lines.
template <int M, int DIR>
__global__ __launch_bounds__(256) void k_fft_rows(cplx<double>* data, size_t nlines, const cplx<double>* twg) {
  constexpr int L = Lanes<M>::value;
  constexpr int NG = 256 / L;
  __shared__ cplx<double> buf[NG * (M + 1)];
  __shared__ cplx<double> tw[M];
  const int tid = threadIdx.x;
  for (int i = tid; i < M; i += 256) tw[i] = twg[i];
  const size_t line0 = (size_t)blockIdx.x * NG;
  for (int i = tid; i < NG * M; i += 256) {
    const int l = i / M, j = i - l * M;
    if (line0 + l < nlines) buf[l * (M + 1) + j] = data[(line0 + l) * M + j];
  }
  __syncthreads();
  const int g = tid / L, lane = tid - g * L;
  if (line0 + g < nlines) fft_group<double, M, DIR, 1>(buf + g * (M + 1), 1, lane, tw);
  __syncthreads();
  for (int i = tid; i < NG * M; i += 256) {
    const int l = i / M, j = i - l * M;
    if (line0 + l < nlines) data[(line0 + l) * M + j] = buf[l * (M + 1) + j];
  }
}

// Strided lines: element j of line x sits at base + x + j*elem_stride; a block handles TX
// consecutive lines (coalesced along x) of one outer index.
template <int M, int DIR, int TX>
__global__ __launch_bounds__(256) void k_fft_cols(cplx<double>* data, size_t elem_stride, size_t outer_stride,
                                                  int inner, const cplx<double>* twg) {
  constexpr int L = Lanes<M>::value;
  constexpr int NG = 256 / L;
  __shared__ cplx<double> buf[TX * (M + 1)];
  __shared__ cplx<double> tw[M];
  const int tid = threadIdx.x;
  for (int i = tid; i < M; i += 256) tw[i] = twg[i];
  const int tiles = inner / TX;
  const int o = blockIdx.x / tiles;
  const int t = blockIdx.x - o * tiles;
  cplx<double>* base = data + (size_t)o * outer_stride + (size_t)t * TX;
  for (int i = tid; i < M * TX; i += 256) {
    const int j = i / TX, x = i - j * TX;
    buf[x * (M + 1) + j] = base[(size_t)j * elem_stride + x];
  }
  __syncthreads();
  const int g = tid / L, lane = tid - g * L;
  for (int x = g; x < TX; x += NG) fft_group<double, M, DIR, 1>(buf + x * (M + 1), 1, lane, tw);
  __syncthreads();
  for (int i = tid; i < M * TX; i += 256) {
    const int j = i / TX, x = i - j * TX;
    base[(size_t)j * elem_stride + x] = buf[x * (M + 1) + j];
  }
}

template <int M, int DIR>
static hipError_t fft3_t(cplx<double>* d, const cplx<double>* tw, hipStream_t s) {
  constexpr int L = Lanes<M>::value;
  constexpr int NG = 256 / L;
  constexpr int TX = M >= 384 ? 8 : (M < 16 ? M : 16);
  const size_t lines = (size_t)M * M;
  hipLaunchKernelGGL((k_fft_rows<M, DIR>), dim3((unsigned)((lines + NG - 1) / NG)), dim3(256), 0, s, d, lines, tw);
  // y lines: element stride M, outer (z) stride M^2
  hipLaunchKernelGGL((k_fft_cols<M, DIR, TX>), dim3(M * (M / TX)), dim3(256), 0, s, d, (size_t)M, (size_t)M * M, M,
                     tw);
  // z lines: element stride M^2, outer (y) stride M
  hipLaunchKernelGGL((k_fft_cols<M, DIR, TX>), dim3(M * (M / TX)), dim3(256), 0, s, d, (size_t)M * M, (size_t)M, M,
                     tw);
  return hipGetLastError();
}

// 2D transforms of `planes` consecutive M x M planes.
template <int M, int DIR>
static hipError_t fft2_t(cplx<double>* d, int planes, const cplx<double>* tw, hipStream_t s) {
  constexpr int L = Lanes<M>::value;
  constexpr int NG = 256 / L;
  constexpr int TX = M >= 384 ? 8 : (M < 16 ? M : 16);
  const size_t lines = (size_t)planes * M;
  hipLaunchKernelGGL((k_fft_rows<M, DIR>), dim3((unsigned)((lines + NG - 1) / NG)), dim3(256), 0, s, d, lines, tw);
  hipLaunchKernelGGL((k_fft_cols<M, DIR, TX>), dim3(planes * (M / TX)), dim3(256), 0, s, d, (size_t)M, (size_t)M * M,
                     M, tw);
  return hipGetLastError();
}

static hipError_t fft3(int M, int dir, cplx<double>* d, const cplx<double>* tw, hipStream_t s) {
#define LS_F3(MM)                                              \
  case MM:                                                     \
    return dir < 0 ? fft3_t<MM, -1>(d, tw, s) : fft3_t<MM, +1>(d, tw, s);
  switch (M) {
    LS_F3(16)
    LS_F3(32)
    LS_F3(64)
    LS_F3(128)
    LS_F3(192)
    LS_F3(256)
    LS_F3(288)
    LS_F3(384)
    LS_F3(512)
    default: return hipErrorInvalidValue;
  }
#undef LS_F3
}

static hipError_t fft2(int M, int dir, cplx<double>* d, int planes, const cplx<double>* tw, hipStream_t s) {
#define LS_F2(MM)                                                                    \
  case MM:                                                                           \
    return dir < 0 ? fft2_t<MM, -1>(d, planes, tw, s) : fft2_t<MM, +1>(d, planes, tw, s);
  switch (M) {
    LS_F2(8)
    LS_F2(16)
    LS_F2(32)
    LS_F2(64)
    LS_F2(96)
    LS_F2(128)
    LS_F2(144)
    LS_F2(192)
    LS_F2(256)
    LS_F2(288)
    LS_F2(384)
    LS_F2(512)
    default: return hipErrorInvalidValue;
  }
#undef LS_F2
}

hipError_t fft2_batched(int M, int dir, cplx<double>* d, int planes, const cplx<double>* tw, hipStream_t s) {
  return fft2(M, dir, d, planes, tw, s);
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

KernelLayout kernel_layout(int n, bool dbl) {
  const size_t c = dbl ? 16 : 8;
  const size_t M = 2 * (size_t)n;
  KernelLayout L;
  L.off_tw = 0;
  L.off_vol = align256(M * c);
  L.off_ff = L.off_vol + align256((size_t)(n + 1) * M * M * c);
  L.total = L.off_ff + align256((size_t)(n + 1) * n * M * c);
  return L;
}

size_t init_ws_bytes(int n) {
  const size_t M = 2 * (size_t)n;
  return 2 * M * M * M * 16 + align256(M * 16);
}

void twiddles(int M, std::vector<double>& re_im) {
  re_im.resize(2 * (size_t)M);
  for (int m = 0; m < M; ++m) {
    // exp(-2 pi i m / M), evaluated from the reduced fraction for accuracy
    const double a = 2.0 * M_PI * (double)m / (double)M;
    re_im[2 * m] = std::cos(a);
    re_im[2 * m + 1] = -std::sin(a);
  }
}

hipError_t green_build(int n, int p, double k, double xg, bool dbl, void* kbuf, void* ws, hipStream_t s) {
  const int M = 2 * n;
  const size_t M3 = (size_t)M * M * M;
  cplx<double>* B = (cplx<double>*)ws;
  cplx<double>* acc = B + M3;
  cplx<double>* twd = acc + M3;
  std::vector<double> tw;
  twiddles(M, tw);
  hipError_t e = hipMemcpyWithStream(twd, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  const KernelLayout KL = kernel_layout(n, dbl);
  char* kb = (char*)kbuf;
  if (dbl) {
    e = hipMemcpyWithStream(kb + KL.off_tw, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice, s);
  } else {
    std::vector<float> twf(tw.begin(), tw.end());
    e = hipMemcpyWithStream(kb + KL.off_tw, twf.data(), twf.size() * sizeof(float), hipMemcpyHostToDevice, s);
  }
  if (e != hipSuccess) return e;

  const int half = p / 2;
  const double R = std::sqrt(3.0) * n;
  const double delta = 2.0 * M_PI / ((double)n * p);
  const int grid = 4096;
  int first = 1;
  for (int s0 = 0; s0 < half; ++s0)
    for (int s1 = 0; s1 < half; ++s1)
      for (int s2 = 0; s2 < half; ++s2) {
        hipLaunchKernelGGL(k_fill_ghat, dim3(grid), dim3(256), 0, s, B, n, half, s0, s1, s2, k, R, delta);
        if ((e = fft3(M, +1, B, twd, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_accum_phase, dim3(grid), dim3(256), 0, s, acc, B, n, p, s0, s1, s2, first);
        first = 0;
      }
  if ((e = fft3(M, -1, acc, twd, s)) != hipSuccess) return e;
  // gm = (8/p^3) (1/M^3) sum (inverse DFT normalisation); the kernel also carries the 1/M^3 of the
  // hot path's unnormalised inverse transform.
  const double m3 = (double)M * M * M;
  const double scale = 8.0 / ((double)p * p * p) / (m3 * m3);
  if (dbl)
    hipLaunchKernelGGL(k_pack_vol<double>, dim3(grid), dim3(256), 0, s, (cplx<double>*)(kb + KL.off_vol), acc, n,
                       scale);
  else
    hipLaunchKernelGGL(k_pack_vol<float>, dim3(grid), dim3(256), 0, s, (cplx<float>*)(kb + KL.off_vol), acc, n,
                       scale);
  if ((e = hipGetLastError()) != hipSuccess) return e;

  // far-field slice kernels, reusing B (n M^2 <= M^3)
  hipLaunchKernelGGL(k_fill_ffslices, dim3(grid), dim3(256), 0, s, B, n, k, xg);
  if ((e = fft2(M, -1, B, n, twd, s)) != hipSuccess) return e;
  const double scale2 = 1.0 / ((double)M * M);
  if (dbl)
    hipLaunchKernelGGL(k_pack_ff<double>, dim3(grid), dim3(256), 0, s, (cplx<double>*)(kb + KL.off_ff), B, n, scale2);
  else
    hipLaunchKernelGGL(k_pack_ff<float>, dim3(grid), dim3(256), 0, s, (cplx<float>*)(kb + KL.off_ff), B, n, scale2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

}  // namespace ls
