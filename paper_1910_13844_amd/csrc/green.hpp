// Green-kernel construction (internal to libls).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

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

}  // namespace ls
