/* A C consumer of libls (no Python, no PyTorch): builds the kernels of one geometry, solves
 * eq. (lipp1) for a set of plane waves and maps the total fields to the detector plane
 * (eq. (lipp2)), using only include/ls.h and the HIP runtime for device memory.
 *
 *   forward_demo <n> <prec 0|1> <kbh> <f.bin> <dirs.bin> <Q> <tol> <out.bin>
 *
 * f.bin: n^3 doubles (the contrast, voxel units); dirs.bin: 3Q doubles.  out.bin receives, per
 * illumination, status, iterations (two int32), the true relative residual (double) and the
 * detector field (n*n complex doubles, converted from the field precision).
 * Exit status 0 on success; a failing call prints its name and ls_strerror. */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "ls.h"

#define LS_TRY(call)                                                                     \
  do {                                                                                   \
    int rc_ = (call);                                                                    \
    if (rc_ != LS_OK) {                                                                  \
      fprintf(stderr, "%s failed: %s (%s)\n", #call, ls_strerror(rc_), ls_last_error()); \
      return 1;                                                                          \
    }                                                                                    \
  } while (0)
#define HIP_TRY(call)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) {                                                              \
      fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));                  \
      return 1;                                                                          \
    }                                                                                    \
  } while (0)

static double* read_doubles(const char* path, size_t count) {
  FILE* fh = fopen(path, "rb");
  if (!fh) return NULL;
  double* v = (double*)malloc(count * sizeof(double));
  size_t got = v ? fread(v, sizeof(double), count, fh) : 0;
  fclose(fh);
  if (got != count) {
    free(v);
    return NULL;
  }
  return v;
}

int main(int argc, char** argv) {
  if (argc != 9) {
    fprintf(stderr, "usage: %s n prec kbh f.bin dirs.bin Q tol out.bin\n", argv[0]);
    return 2;
  }
  const int n = atoi(argv[1]), prec = atoi(argv[2]), Q = atoi(argv[6]);
  const double kbh = atof(argv[3]), tol = atof(argv[7]);
  if (n < 8 || (prec != LS_C64 && prec != LS_C128) || Q < 1) return 2;
  const size_t N = (size_t)n * n * n, real_sz = prec == LS_C128 ? 8 : 4, cplx_sz = 2 * real_sz;
  double* f64 = read_doubles(argv[4], N);
  double* dirs = read_doubles(argv[5], 3 * (size_t)Q);
  if (!f64 || !dirs) {
    fprintf(stderr, "cannot read inputs\n");
    return 2;
  }

  ls_geom g = {n, 4, kbh, (double)n, prec, 0};
  size_t kb = 0, iwb = 0, wsb = 0, ffb = 0;
  LS_TRY(ls_kernel_bytes(&g, &kb));
  LS_TRY(ls_init_workspace_bytes(&g, &iwb));
  void *kbuf = NULL, *iws = NULL;
  HIP_TRY(hipMalloc(&kbuf, kb));
  HIP_TRY(hipMalloc(&iws, iwb));
  ls_ctx* ctx = NULL;
  LS_TRY(ls_green_init(&g, kbuf, kb, iws, iwb, NULL, &ctx));
  HIP_TRY(hipFree(iws));

  /* contrast in the field precision */
  void* f_host = malloc(N * real_sz);
  for (size_t i = 0; i < N; ++i) {
    if (prec == LS_C128)
      ((double*)f_host)[i] = f64[i];
    else
      ((float*)f_host)[i] = (float)f64[i];
  }
  void *f = NULL, *u = NULL, *y = NULL, *ws = NULL;
  HIP_TRY(hipMalloc(&f, N * real_sz));
  HIP_TRY(hipMemcpy(f, f_host, N * real_sz, hipMemcpyHostToDevice));
  HIP_TRY(hipMalloc(&u, (size_t)Q * N * cplx_sz));
  HIP_TRY(hipMalloc(&y, (size_t)Q * n * n * cplx_sz));
  LS_TRY(ls_workspace_bytes(ctx, Q, LS_OP_FORWARD, &wsb));
  LS_TRY(ls_workspace_bytes(ctx, Q, LS_OP_FARFIELD, &ffb));
  HIP_TRY(hipMalloc(&ws, wsb > ffb ? wsb : ffb));

  ls_solve_opts opts = {tol, 1000, 3};
  ls_solve_info* info = (ls_solve_info*)calloc((size_t)Q, sizeof(ls_solve_info));
  LS_TRY(ls_forward(ctx, f, Q, dirs, u, &opts, info, ws, wsb, NULL));
  LS_TRY(ls_farfield(ctx, f, u, Q, y, ws, ffb, NULL));
  HIP_TRY(hipDeviceSynchronize());

  const size_t ny = (size_t)Q * n * n;
  void* y_host = malloc(ny * cplx_sz);
  HIP_TRY(hipMemcpy(y_host, y, ny * cplx_sz, hipMemcpyDeviceToHost));
  FILE* out = fopen(argv[8], "wb");
  if (!out) return 2;
  for (int q = 0; q < Q; ++q) {
    fwrite(&info[q].status, sizeof(int32_t), 1, out);
    fwrite(&info[q].iters, sizeof(int32_t), 1, out);
    fwrite(&info[q].relres_true, sizeof(double), 1, out);
    for (size_t i = 0; i < (size_t)2 * n * n; ++i) {
      const size_t k = (size_t)q * 2 * n * n + i;
      const double v = prec == LS_C128 ? ((double*)y_host)[k] : (double)((float*)y_host)[k];
      fwrite(&v, sizeof(double), 1, out);
    }
  }
  fclose(out);
  printf("forward_demo: n=%d prec=%d Q=%d iterations", n, prec, Q);
  for (int q = 0; q < Q; ++q) printf(" %d", info[q].iters);
  printf("\n");

  ls_ctx_destroy(ctx);
  hipFree(ws);
  hipFree(y);
  hipFree(u);
  hipFree(f);
  hipFree(kbuf);
  free(y_host);
  free(info);
  free(f_host);
  free(f64);
  free(dirs);
  return 0;
}
