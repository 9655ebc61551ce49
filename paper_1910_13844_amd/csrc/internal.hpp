// Internal structures shared by the kernels and the host engine (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ls {

// Per-slot vectors.  A slot is one right-hand side (one illumination) of a batched solve.
enum Vec : int {
  V_X = 0,   // iterate / solution (caller-owned u)
  V_R = 1,   // residual
  V_RH = 2,  // shadow residual
  V_P = 3,
  V_V = 4,
  V_S = 5,
  V_T = 6,
  V_SPEC = 7,  // x-spectrum scratch: [2n kx][nz][n y]
  V_B = 8,     // stored right-hand side (null: plane wave)
  V_AUX = 9,   // detector-plane buffer or other per-slot I/O
  V_SPE = 10,  // (y,z)-convolved x-spectrum by ky class, [c][2n kx][n z][2n/C]; spans V_SPE and V_SPO
  V_SPO = 11,  // second half of that region (class 1 of the parity split)
  V_COUNT = 12
};

struct SlotDesc {
  void* vec[V_COUNT];
  const void* f;  // real potential, N values (float for c64, double for c128)
  double d[3];    // plane-wave direction (unit vector)
  double k;       // k_b h
  int32_t pad[2];
};

// Solver status codes kept on the device.
enum Status : int32_t {
  ST_RUN = 0,     // iterating
  ST_HALF = 1,    // converged on s; the update applies x += alpha p
  ST_CHECK = 2,   // recursion finished (converged or out of iterations): true residual pending
  ST_OK = 3,      // done, true residual within tolerance
  ST_MAXIT = 4,   // done, not converged within maxit
  ST_BREAK = 5,   // done, breakdown not recovered
  ST_NONFIN = 6,  // done, non-finite values
  ST_IDLE = 7,    // slot unused
  ST_INIT = 8     // admitted: initial residual pending
};

struct SlotState {
  double rho[2], rho_prev[2], alpha[2], omega[2], beta[2];
  double nb, rr, nrh, relres, relres_true, tol;
  double brk;  // breakdown threshold: restart when |rho| <= brk ||rh|| ||r||
  int32_t status, iters, matvecs, restarts, restart_flag, maxit, max_restarts, reason;
  uint64_t t_start, t_done;  // device steady clock: first pass of the slot, final state reached
};

// Partial sums per block: up to 4 complex FP64 numbers.
constexpr int PART_K = 4;

// Prologue of the forward x-pass (what is transformed).
enum Pro : int {
  PRO_F_VEC = 0,   // f . vec[sel]
  PRO_F_B = 1,     // f . b (plane wave or stored)
  PRO_P = 2,       // p = r + beta (p - omega v), f . p  (restart: p = r, rh = r)
  PRO_S = 3,       // s = r - alpha v, f . s, partial ||s||^2
  PRO_VEC = 4,     // vec[sel]
  PRO_CONJ_VEC = 5 // conj(vec[sel])
};

// Epilogue of the inverse x-pass (g = the convolution result at a voxel).
enum Epi : int {
  EPI_STORE = 0,  // vec[sel] = g
  EPI_AXV = 1,    // v = p - g, partial <rh, v>
  EPI_AXT = 2,    // t = s - g, partials <t, s>, ||t||^2
  EPI_R0 = 3,     // x = b, r = rh = g, partials ||g||^2, ||b||^2
  EPI_TRUE = 4,   // r = b - x + g, partial ||r||^2
  EPI_AX = 5,     // vec[sel2] = vec[sel] - g
  EPI_R0X = 6     // warm start (x given): r = rh = b - x + g, partials ||r||^2, ||b||^2
};

struct PassArgs {
  const SlotDesc* desc;
  SlotState* st;
  double* part;      // [slot][PART_STRIDE][PART_K][2]
  int part_stride;   // blocks per slot
  int nslots;
  int nz;            // rows along z (n for volumes, 1 for detector planes)
  uint32_t mask;     // slot runs iff (1 << status) & mask
  int mode;          // prologue / epilogue
  int sel, sel2;
  int spec;          // vector holding the x-spectrum read or written by the pass
  int spec2;         // k_xinv: second half to combine (odd ky), or -1
  const void* tw;    // twiddle table exp(-2 pi i m / 2n), m < 2n
  const void* kern;  // Fourier kernel (pass-specific layout)
};

}  // namespace ls
