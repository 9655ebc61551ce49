/* libls: Lippmann-Schwinger forward model, far field and data-term gradient on MI355X (gfx950).
 *
 * Pham, Soubies, Ayoub, Lim, Psaltis, Unser, "Three-Dimensional Optical Diffraction Tomography
 * with Lippmann-Schwinger Model" (arXiv 1910.13844).
 *
 * Conventions shared by every call
 * --------------------------------
 * Units: voxel units, h = 1.  kbh = k_b h with k_b = 2 pi eta_b / lambda0; the contrast passed
 *   in is f~ = f h^2 = (2 pi h / lambda0)^2 (eta^2 - eta_b^2) (Section "Continuous-Domain
 *   Formulation").  x_Gamma is given in voxels.
 * Grid: Omega_n = [[-n/2+1, n/2]]^3 (Theorem 1).  Volume arrays are row-major [z][y][x], x fastest;
 *   array index i holds the signed position i - n/2 + 1.  Detector arrays are [y][x] (m = n) at the
 *   same lateral positions.  Batches add a leading illumination index [Q].
 * Types: complex = interleaved (re, im) in the path's precision: LS_C64 -> float, LS_C128 ->
 *   double; real arrays (f, gradients) use float / double accordingly.
 * Memory: every array pointer is DEVICE memory owned by the caller unless marked [host].  The
 *   library allocates no device memory: device scratch comes from caller-provided workspaces whose
 *   sizes the *_bytes queries return.  A workspace must not be used by two calls at once.
 * Streams: `stream` is a hipStream_t (NULL = default stream).  Calls enqueue work on it and return;
 *   calls that produce [host] outputs (solve information, loss) synchronise that stream first.
 * Errors: 0 on success, a negative LS_ERR_* code otherwise; arguments are validated before
 *   anything is enqueued.  The library never aborts or throws across this interface.  Per-
 *   illumination non-convergence is not a call failure: it is reported in ls_solve_info.status.
 */
#ifndef LS_H_
#define LS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LS_OK 0
#define LS_ERR_ARG (-1)       /* invalid argument (sizes, Nyquist condition, null pointers) */
#define LS_ERR_WORKSPACE (-2) /* workspace or kernel buffer too small */
#define LS_ERR_UNSUPPORTED (-3) /* grid size / precision combination not built */
#define LS_ERR_HIP (-4)       /* a HIP runtime call failed; see ls_last_error() */

#define LS_C64 0  /* complex64 fields, FP64 reductions and Krylov scalars */
#define LS_C128 1 /* complex128 throughout */

/* Geometry of one problem (Theorem 1, Proposition 2, Section on G~). */
typedef struct {
  int32_t n;    /* voxels per side; supported: 8, 16, 32, 64, 96, 128, 144, 192, 256 (both precisions) */
  int32_t p;    /* Theorem 1 padding factor, even, >= 2 (p = 4 recommended); only the 2n grid is stored */
  double kbh;   /* k_b h; must satisfy 0 < kbh < pi (Nyquist condition of Theorem 1) */
  double xg;    /* detector plane position x_Gamma / h; must exceed n/2 (plane outside Omega) */
  int32_t prec; /* LS_C64 or LS_C128 */
  int32_t reserved;
} ls_geom;

typedef struct {
  double tol;           /* stop when ||b - A x|| / ||b|| <= tol (recursive residual, re-checked in FP64) */
  int32_t maxit;        /* iteration cap per illumination */
  int32_t max_restarts; /* restarts allowed after breakdown or a failed true-residual check */
  int32_t x0_mode;      /* initial guess of ls_forward / ls_forward_uin: 0 x0 = u_in (the incident
                           field), 1 x0 = the contents of u on entry (warm start, e.g. the fields of
                           the previous reconstruction iterate); other calls use x0 = b */
  int32_t reserved;     /* 0 */
  double breakdown;     /* breakdown threshold eps of the restart test |<rh, r>| <= eps ||rh|| ||r|| (the
                           method's safeguard against a vanishing rho; restart with rh = r, p = v = 0).
                           0 = the unit roundoff of the field precision (default); otherwise 0 < eps < 1.
                           The test runs from the second iteration on (at the first, rh = r).
                           LS_ERR_ARG if negative, >= 1 or not finite. */
} ls_solve_opts;

typedef struct {
  int32_t status;      /* 0 converged, 1 iteration cap, 2 breakdown not recovered, 3 non-finite */
  int32_t iters;       /* BiCGSTAB iterations */
  int32_t matvecs;     /* applications of A = I - G diag f */
  int32_t restarts;
  double relres_rec;   /* last recursive relative residual */
  double relres_true;  /* ||b - A x|| / ||b|| recomputed from x (FP64 accumulation) */
  double time_ms;      /* device-clock time from the illumination's first pass (its initial
                          residual) to its final state; -1 if it has not reached one */
} ls_solve_info;

typedef struct ls_ctx ls_ctx;     /* immutable after ls_green_init; host-side object */
typedef struct ls_batch ls_batch; /* slot pool for continuous batching; host-side object */

/* Human-readable text for an error code; ls_last_error() gives the last HIP error text. */
const char* ls_strerror(int code);
const char* ls_last_error(void);

/* Sizes of the caller-allocated buffers of ls_green_init.  kernel: Fourier-domain volume kernel
 * and far-field slice kernels plus twiddles (kept for the lifetime of the context); init
 * workspace: FP64 scratch needed only during ls_green_init. */
int ls_kernel_bytes(const ls_geom* g, size_t* bytes);
int ls_init_workspace_bytes(const ls_geom* g, size_t* bytes);

/* Builds the Fourier-domain Green kernels for geometry g (Proposition 2; Section on G~).
 *   ghat_m = F_{2n}(gm),  gm[k] = (8/p^3) sum_{s in [[0,p/2-1]]^3} F^{-1}_{2n}(ghat_t[(p/2).-s])[k]
 *            e^{-2 i pi k.s/(np)},  ghat_t the transform of the Green function truncated at
 *            sqrt(3) L (eqs. (GreenL), (GreenL2));
 *   far-field slice kernels: 2n-padded 2D DFTs of g(., x_Gamma - z_k) sampled on the voxel grid.
 * All in FP64, rounded once to the path precision.  kbuf (>= ls_kernel_bytes) must stay valid
 * while the context is used; ws (>= ls_init_workspace_bytes) may be reused after return.
 * Synchronises `stream`.  *out receives a host-side context (free with ls_ctx_destroy). */
int ls_green_init(const ls_geom* g, void* kbuf, size_t kbuf_bytes, void* ws, size_t ws_bytes, void* stream,
                  ls_ctx** out);
void ls_ctx_destroy(ls_ctx* ctx);

#define LS_OP_FORWARD 0  /* ls_forward */
#define LS_OP_FARFIELD 1 /* ls_farfield, ls_farfield_adj */
#define LS_OP_GRAD 2     /* ls_grad, ls_vjp */
#define LS_OP_APPLY 3    /* ls_apply_G, ls_apply_A */
#define LS_OP_PROX 4     /* ls_prox_tv, ls_tv_value (Q is ignored) */
#define LS_OP_INCIDENT 5 /* ls_incident_field */
/* Workspace needed to process Q illuminations of operation `op` in one group.  Calls accept any
 * workspace that fits at least one illumination and process the batch in groups. */
int ls_workspace_bytes(const ls_ctx* ctx, int32_t Q, int32_t op, size_t* bytes);

/* out_q = G v_q for Q volumes v [Q][N] (Theorem 1 / Proposition 2). */
int ls_apply_G(const ls_ctx* ctx, const void* v, void* out, int32_t Q, void* ws, size_t ws_bytes, void* stream);
/* out_q = v_q - G (f . v_q): the operator of eq. (lipp1). */
int ls_apply_A(const ls_ctx* ctx, const void* f, const void* v, void* out, int32_t Q, void* ws, size_t ws_bytes,
               void* stream);

/* Forward solve, eq. (lipp1): u_q = (I - G diag f)^{-1} u_in,q for plane waves
 * u_in,q(x) = exp(i kbh d_q . x), d_q = dirs[3q..3q+2] [host] (unit vectors, (x, y, z) order).
 * BiCGSTAB (van der Vorst) with x0 = u_in, FP64 inner products and scalars.  u: out [Q][N].
 * info: [host] Q entries (may be NULL).  Synchronises `stream`. */
int ls_forward(const ls_ctx* ctx, const void* f, int32_t Q, const double* dirs, void* u, const ls_solve_opts* opts,
               ls_solve_info* info, void* ws, size_t ws_bytes, void* stream);

/* ls_forward followed by the far field of every solution, y_q = G~ (f . u_q) (eq. (lipp2), P = I):
 * the solve of one illumination and its detector field.  Equal bit for bit to ls_forward then
 * ls_farfield, without the far field's own x-forward pass: the solver's final true-residual check
 * already transformed f . u_q.  u: out [Q][N]; y: out [Q][m][m]; ws as for ls_forward. */
int ls_forward_farfield(const ls_ctx* ctx, const void* f, int32_t Q, const double* dirs, void* u, void* y,
                        const ls_solve_opts* opts, ls_solve_info* info, void* ws, size_t ws_bytes, void* stream);

/* ls_forward_farfield for callers that cannot allocate device memory (serving loops and harnesses
 * that must not call the allocator): the same computation, its scratch taken from a fixed device
 * array of LS_SCRATCH_BYTES that the library holds on each device it runs on until the process ends
 * (no workspace argument; no allocation in the call).  Like ls_forward it waits on `stream` between
 * groups of iterations to read the solver states, so it cannot be recorded under stream capture.
 * The batch runs in groups of as many illuminations as fit that array.  Every call on one device
 * shares the array, which keeps the last call's contents (each call writes every part it reads
 * before reading it): calls that overlap on a device (other threads or streams) race and must be
 * serialised by the caller.
 * Errors: LS_ERR_WORKSPACE when one illumination of the context's grid needs more scratch than
 * LS_SCRATCH_BYTES (for complex64 up to n = 128; complex128 up to n = 96); otherwise as
 * ls_forward_farfield. */
#define LS_SCRATCH_BYTES (256u * 1024u * 1024u)
int ls_forward_farfield_noalloc(const ls_ctx* ctx, const void* f, int32_t Q, const double* dirs, void* u, void* y,
                                const ls_solve_opts* opts, ls_solve_info* info, void* stream);

/* Far field, eq. (lipp2) with P = I: y_q = G~ (f . u_q) on the detector plane x3 = x_Gamma,
 * a sum over z-slices of 2D aperiodic convolutions with g.  u: [Q][N]; y: out [Q][m][m]. */
int ls_farfield(const ls_ctx* ctx, const void* f, const void* u, int32_t Q, void* y, void* ws, size_t ws_bytes,
                void* stream);
/* Transpose of G~ (no conjugation unless conj != 0, then applied to conj(r)): out = G~^T r,
 * r: [Q][m][m], out: [Q][N]. */
int ls_farfield_adj(const ls_ctx* ctx, const void* r, int32_t conj, int32_t Q, void* out, void* ws, size_t ws_bytes,
                    void* stream);

/* Vector-Jacobian product of y_q(f) = G~ diag(f) u_q(f) (Algorithm 1, gradient step):
 *   grad = sum_q Re(J_q^* gy_q),  gy = dL/dRe(y) + i dL/dIm(y)  [Q][m][m],
 * evaluated as Re(u_q . w_q) with (I - G diag f) w_q = G~^T conj(gy_q) (one more solve per view).
 * u: the forward fields [Q][N].  grad: out [N] real.  info: [host] Q entries (adjoint solves). */
int ls_vjp(const ls_ctx* ctx, const void* f, const void* u, int32_t Q, const void* gy, void* grad,
           const ls_solve_opts* opts, ls_solve_info* info, void* ws, size_t ws_bytes, void* stream);

/* Data term of eq. (prob) and its gradient (Algorithm 1, gradient step):
 *   loss = sum_q ||H_q(f) - y_meas,q||^2 / (2 ||y_meas,q||^2),
 *   grad = sum_q Re(J_q^* (H_q(f) - y_meas,q)) / ||y_meas,q||^2.
 * y_meas: [Q][m][m]; grad: out [N]; loss: [host]; info: [host] 2Q entries (forward, then adjoint). */
int ls_grad(const ls_ctx* ctx, const void* f, int32_t Q, const double* dirs, const void* y_meas, void* grad,
            double* loss, const ls_solve_opts* opts, ls_solve_info* info, void* ws, size_t ws_bytes, void* stream);

/* Building blocks of the gradient for callers that schedule the solves themselves (the
 * continuous-batching loop):
 *   ls_residual: FP64 sums stats[2q] = ||y_q - y_meas,q||^2, stats[2q+1] = ||y_meas,q||^2, and
 *     r_q = y_q - y_meas,q (weighted == 0) or r_q = (y_q - y_meas,q) / ||y_meas,q||^2 (weighted != 0:
 *     the gradient of the data term with respect to y_q, dL/dRe(y) + i dL/dIm(y)); loss (device double,
 *     may be NULL) = the data term of eq. (prob), sum_q stats[2q] / (2 stats[2q+1]), summed in q order.
 *     y, y_meas, r: [Q][m][m] device (r may alias y); stats: [2Q] device doubles.  The weighted form
 *     needs ||y_meas,q|| > 0.
 *   ls_grad_accumulate: grad[i] (+)= sum_q w_q Re(u_q[i] wb_q[i]) (Algorithm 1, gradient step, with
 *     wb_q solving (I - G diag f) wb_q = G~^T conj(r_q)); w_q = 1 / stats[2q+1] when stats is given,
 *     else 1.  Summed over q in index order in FP64.  u, wb: [Q][N]; grad: [N] real, overwritten when
 *     accumulate == 0, added to otherwise. */
int ls_residual(const ls_ctx* ctx, const void* y, const void* y_meas, int32_t Q, int32_t weighted, void* r,
                double* stats, double* loss, void* stream);
int ls_grad_accumulate(const ls_ctx* ctx, const void* u, const void* wb, int32_t Q, const double* stats,
                       void* grad, int32_t accumulate, void* stream);

/* Continuous batching (slot pool).  A batch holds `nslots` independent solves of eq. (lipp1) on
 * one context (one grid size); each slot has its own potential, right-hand side and output.
 * Slots are admitted and harvested between steps while the others keep iterating, so requests
 * that arrive while others run share the same kernel launches.
 *   ls_batch_bytes:   workspace for nslots slots.
 *   ls_batch_create:  host object over the caller's workspace; all slots idle.
 *   ls_batch_admit:   start a solve in an idle slot: f [N], either dir [host, 3] (plane wave) or
 *                     b [N] (stored right-hand side, device), and the output x [N] (device).
 *   ls_batch_step:    run up to `iters` iterations of every running slot (and pending true-
 *                     residual checks), then synchronise and refresh the slot states.
 *   ls_batch_poll:    [host] state per slot (0 idle, 1 running, 2 done) and solve info.
 *   ls_batch_release: mark a done slot idle again. */
int ls_batch_bytes(const ls_ctx* ctx, int32_t nslots, size_t* bytes);
int ls_batch_create(const ls_ctx* ctx, int32_t nslots, void* ws, size_t ws_bytes, const ls_solve_opts* opts,
                    ls_batch** out);
int ls_batch_admit(ls_batch* b, int32_t slot, const void* f, const double* dir, const void* rhs, void* x,
                   void* stream);
int ls_batch_step(ls_batch* b, int32_t iters, void* stream);
int ls_batch_poll(const ls_batch* b, int32_t* state, ls_solve_info* info);
int ls_batch_release(ls_batch* b, int32_t slot);
void ls_batch_destroy(ls_batch* b);

/* Incident fields from measured detector fields (Section "Computation of the 3D Incident Field",
 * angular spectrum with tilt transfer).  y_in: device [Q][n][n] complex (field precision), the field
 * on the detector plane x3 = x_Gamma sampled on the lateral voxel grid ([y][x], positions i - n/2 + 1).
 * ktilde: [host] Q x 2 lateral wave-vector components (k~_x, k~_y) in radians per voxel, read when
 * tilt != 0.  uin: out [Q][N].  For each slice z: u_in = exp(i x~.k~) IDFT2( DFT2(y_in exp(-i x~.k~))
 * exp(-i (x_Gamma - z) sqrt(kbh^2 - |w + k~|^2)) ), periodic 2D DFTs over the n x n grid, evanescent
 * components (|w + k~| > kbh) dropped; tilt = 0 propagates y_in itself (k~ = 0).  FP64 throughout,
 * rounded once.  ws >= ls_workspace_bytes(ctx, Qg, LS_OP_INCIDENT) for some group Qg >= 1 (the call
 * processes the batch in groups).  Errors: LS_ERR_ARG (null pointers, non-finite tilt),
 * LS_ERR_WORKSPACE. */
int ls_incident_field(const ls_ctx* ctx, const void* y_in, const double* ktilde, int32_t Q, int32_t tilt, void* uin,
                      void* ws, size_t ws_bytes, void* stream);
/* Forward solve, eq. (lipp1), with stored incident fields: as ls_forward with b = x0 = uin[q]
 * (device [Q][N], e.g. from ls_incident_field) instead of plane waves.  uin must not alias u. */
int ls_forward_uin(const ls_ctx* ctx, const void* f, int32_t Q, const void* uin, void* u, const ls_solve_opts* opts,
                   ls_solve_info* info, void* ws, size_t ws_bytes, void* stream);

/* Detector-side operators of eq. (lipp2) (Sections "Green's Function Discretization for the
 * Measurements" and "Free-Space Propagation and Pupil Function"), on m x m detector fields
 * [Q][m][m] complex (field precision, device), pixel spacing h, grids centred (pixel a at lateral
 * position a - m/2 + 1).  FP64 internally, rounded once.
 * ls_detector_bytes: workspace for the calls below with this m.
 * ls_farfield_wide: y = G~_m (f . u) on a camera of m >= n pixels (m - n even): the slice sum of
 *   2D linear convolutions with the untruncated g, by DFTs of size M >= m + n - 1 (M from 8, 16,
 *   32, 64, 96, 128, 144, 192, 256, 288, 384, 512, else LS_ERR_UNSUPPORTED).  m = n equals ls_farfield.
 * ls_farfield_wide_adj: out [Q][N] = G~_m^T r (or G~_m^T conj(r) when conj != 0), the transpose.
 * ls_pupil: out = crop_m IDFT_2m( p . DFT_2m(pad y) ), p(w) = 1{|w| <= na kbh} exp(i dz sqrt(kbh^2 -
 *   |w|^2)) (ideal pupil of numerical aperture na relative to the background index, propagation
 *   over dz voxels); adjoint != 0 applies conj(p).  2m must be one of the DFT sizes above.
 * ls_decimate: detector sampling h' = q h: out [Q][m/q][m/q] keeps every q-th pixel (the kept set
 *   contains the pixel at lateral position 0); transpose != 0 maps [Q][m/q][m/q] back to [Q][m][m]
 *   with zeros elsewhere.  m % q == 0; out must not alias y.
 * Errors: LS_ERR_ARG (null pointers, m < n or m - n odd for the far field, non-finite na/dz),
 * LS_ERR_UNSUPPORTED (DFT size), LS_ERR_WORKSPACE. */
int ls_detector_bytes(const ls_ctx* ctx, int32_t m, size_t* bytes);
int ls_farfield_wide(const ls_ctx* ctx, int32_t m, const void* f, const void* u, int32_t Q, void* y, void* ws,
                     size_t ws_bytes, void* stream);
int ls_farfield_wide_adj(const ls_ctx* ctx, int32_t m, const void* r, int32_t conj, int32_t Q, void* out, void* ws,
                         size_t ws_bytes, void* stream);
int ls_pupil(const ls_ctx* ctx, int32_t m, const void* y, int32_t Q, double na, double dz, int32_t adjoint, void* out,
             void* ws, size_t ws_bytes, void* stream);
int ls_decimate(const ls_ctx* ctx, int32_t m, int32_t q, const void* y, int32_t Q, void* out, int32_t transpose,
                void* stream);
/* Gradient for a volume right-hand side (the Jacobian-adjoint step of Algorithm 1 behind any detector
 * chain): grad [N] real = sum_q Re(u_q . w_q), (I - G diag f) w_q = b_q.  With b_q = G~^T conj(B^* gy_q)
 * for a detector chain B this is Re(J^* gy) of the chained model.  ws as for LS_OP_GRAD. */
int ls_vjp_rhs(const ls_ctx* ctx, const void* f, const void* u, int32_t Q, const void* b, void* grad,
               const ls_solve_opts* opts, ls_solve_info* info, void* ws, size_t ws_bytes, void* stream);

/* Reconstruction step (Algorithm 1, Section "Optimization").  Fields are real [N] arrays of the
 * context's precision (float for LS_C64, double for LS_C128), device memory owned by the caller.
 *
 * ls_prox_tv: x = prox of lam TV + i_{>=0} at z = v - gamma d (d may be NULL: z = v), i.e.
 *   argmin_x 1/2 ||x - z||^2 + lam TV(x) (+ indicator of x >= 0 when nonneg != 0),
 * with TV isotropic over forward differences (zero across the far faces of the grid), by `iters`
 * steps of fast gradient projection on the dual (step 1/(12 lam)); lam = 0 or iters = 0 give the
 * projection of z.  For the prox step of Algorithm 1 pass lam = gamma_k tau.  x may alias v or d.
 * ws >= ls_workspace_bytes(ctx, 1, LS_OP_PROX).  Errors: LS_ERR_ARG (null pointer, negative or
 * non-finite lam, non-finite gamma, iters < 0), LS_ERR_WORKSPACE.
 * ls_fbs_extrapolate: v_out = f + beta (f - f_prev), the extrapolation of Algorithm 1 with
 *   beta = (a_k - 1) / a_{k+1}; v_out may alias f or f_prev.
 * ls_tv_value: [host] out = TV(x), accumulated in FP64 in a fixed order; synchronises `stream`. */
int ls_prox_tv(const ls_ctx* ctx, const void* v, const void* d, double gamma, double lam, int32_t iters,
               int32_t nonneg, void* x, void* ws, size_t ws_bytes, void* stream);
int ls_fbs_extrapolate(const ls_ctx* ctx, const void* f, const void* f_prev, double beta, void* v_out, void* stream);
int ls_tv_value(const ls_ctx* ctx, const void* x, double* out, void* ws, size_t ws_bytes, void* stream);

/* Timing hook: enqueues `reps` launches of one pass of the solver iteration over Q slots of a
 * LS_OP_FORWARD workspace, so a single kernel can be timed in isolation (the computation of the
 * iteration, not a separate code path).  pass: 0 x-forward with the p-update prologue,
 * 1 (y,z) plane convolution, 2 x-inverse with the v = p - G(f p) epilogue, 3 vector update.
 * f [N] and u [Q][N] as for ls_forward; the workspace contents are overwritten. */
int ls_profile_pass(const ls_ctx* ctx, const void* f, void* u, int32_t pass, int32_t Q, int32_t reps, void* ws,
                    size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LS_H_ */
