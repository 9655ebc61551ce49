// Green-kernel construction (internal to libls).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include <vector>

#include "cplx.hpp"

namespace ls {

struct KernelLayout {
  size_t off_tw;   // twiddles exp(-2 pi i m / 2n), m < 2n, path precision
  size_t off_vol;  // volume kernel [n+1][2n][2n]
  size_t off_ff;   // far-field kernel [n+1][n][2n]
  size_t total;
};

KernelLayout kernel_layout(int n, bool dbl);
size_t init_ws_bytes(int n);
hipError_t green_build(int n, int p, double k, double xg, bool dbl, void* kbuf, void* ws, hipStream_t s);

// FP64 tools shared with the incident-field propagation: twiddles exp(-2 pi i m / M), m < M, as
// interleaved (re, im); unnormalised 2D DFTs (sign dir) of `planes` contiguous M x M planes, with
// the twiddle table of length M in device memory.
void twiddles(int M, std::vector<double>& re_im);
hipError_t fft2_batched(int M, int dir, cplx<double>* d, int planes, const cplx<double>* tw, hipStream_t s);

}  // namespace ls
