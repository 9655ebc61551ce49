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
hipError_t launch_residual(bool dbl, int m, const void* y, const void* ymeas, int Q, bool weighted, void* r,
                           double* stats, double* loss, hipStream_t s);

// reconstruction step (recon.hip)
hipError_t launch_prox_init(bool dbl, const void* v, const void* d, double gamma, void* z, void* p, void* r,
                            size_t N, hipStream_t s);
hipError_t launch_prox_primal(bool dbl, const void* b, const void* q, double lam, int nonneg, void* x, int n,
                              hipStream_t s);
hipError_t launch_prox_dual(bool dbl, const void* x, void* p, void* r, double step, double beta, int n, hipStream_t s);
hipError_t launch_extrapolate(bool dbl, const void* f, const void* fp, double beta, void* out, size_t N,
                              hipStream_t s);
hipError_t launch_tv_value(bool dbl, const void* x, int n, double* part, double* out, hipStream_t s);
int tv_partial_blocks(size_t N);

// incident field from detector fields (incident.hip)
hipError_t launch_inc_demod(bool dbl, const void* y, const double* kt, int tilt, void* A, int n, int Q,
                            hipStream_t s);
hipError_t launch_inc_prop(const void* A, const double* kt, int tilt, double k, double xg, void* B, int n, int Q,
                           hipStream_t s);
hipError_t launch_inc_mod(bool dbl, const void* B, const double* kt, int tilt, void* u, int n, int Q, hipStream_t s);

// detector-side operators (detector.hip)
hipError_t launch_det_kernel(void* K, int n, int M, int s, double k, double xg, hipStream_t st);
hipError_t launch_det_pad_vol(bool dbl, const void* f, const void* u, void* V, int n, int M, hipStream_t st);
hipError_t launch_det_pad2(bool dbl, const void* y, void* P, int m, int M, int Q, int cj, hipStream_t st);
hipError_t launch_det_mulsum(const void* K, const void* V, void* Y, int n, int M, hipStream_t st);
hipError_t launch_det_mulT(const void* K, const void* R, void* V, int n, int M, hipStream_t st);
hipError_t launch_det_crop(bool dbl, const void* Y, void* out, int m, int M, int Q, double scale, hipStream_t st);
hipError_t launch_det_pupil(void* P, int M, int Q, double k, double wc, double dz, int adjoint, hipStream_t st);
hipError_t launch_decimate(bool dbl, const void* y, void* out, int m, int q, int s, int Qn, int transpose,
                           hipStream_t st);

inline int ty_of(int n) { return n < 16 ? n : 16; }
inline int blocks_per_slot(int n, int nz) { return nz * (n / ty_of(n)); }

}  // namespace ls
