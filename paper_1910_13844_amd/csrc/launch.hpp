// Host-side launchers of the device kernels (internal to libls).
#pragma once
#include "internal.hpp"

namespace ls {

bool fused_supported(int n, bool dbl);

// x-forward pass, (y,z) convolution, x-inverse pass, far-field passes.
hipError_t launch_xfwd(bool dbl, int n, const PassArgs& a, hipStream_t s);
hipError_t launch_xinv(bool dbl, int n, const PassArgs& a, hipStream_t s);
hipError_t launch_yz(bool dbl, int n, const PassArgs& a, hipStream_t s);
hipError_t launch_ff(bool dbl, int n, const PassArgs& a, hipStream_t s);
hipError_t launch_ffT(bool dbl, int n, const PassArgs& a, hipStream_t s);
hipError_t launch_update(bool dbl, int n, const PassArgs& a, hipStream_t s);

enum Scalar : int { SC_INIT = 0, SC_ALPHA = 1, SC_OMEGA = 2, SC_BETA = 3, SC_FINAL = 4 };
hipError_t launch_scalar(int kind, bool dbl, const PassArgs& a, hipStream_t s);

// gradient helpers
hipError_t launch_grad_accum(bool dbl, int n, const SlotDesc* desc, const double* w, int nslots, int sel_u,
                             int sel_w, void* grad, int accumulate, hipStream_t s);
hipError_t launch_grad_sum(bool dbl, const void* u, const void* wb, int Q, size_t N, const double* stats, void* grad,
                           int accumulate, hipStream_t s);
hipError_t launch_convert(bool dbl, const double* src, void* dst, size_t N, hipStream_t s);
hipError_t launch_residual(bool dbl, int m, const void* y, const void* ymeas, int Q, void* r, double* stats,
                           hipStream_t s);

inline int ty_of(int n) { return n < 16 ? n : 16; }
inline int blocks_per_slot(int n, int nz) { return nz * (n / ty_of(n)); }

}  // namespace ls
