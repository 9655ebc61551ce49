// C ABI of libls and the host engine behind it (batched BiCGSTAB over slots, far field,
// gradient, slot pools).  Host code only; all arithmetic runs in the kernels of kernels.hip and
// green.hip.
#include "ls.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "green.hpp"
#include "launch.hpp"

using namespace ls;

struct ls_ctx {
  ls_geom g;
  bool dbl;
  int n;
  size_t csz;  // bytes per complex
  size_t N;    // n^3
  char* kbuf;
  void* tw;
  void* kvol;
  void* kff;
  double clk_khz;  // rate of the device steady clock (ticks per ms)
};

namespace {

thread_local std::string g_last_error;

int hip_fail(hipError_t e, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  return LS_ERR_HIP;
}

#define HIPCHK(x)                                        \
  do {                                                   \
    hipError_t _e = (x);                                 \
    if (_e != hipSuccess) return hip_fail(_e, #x);       \
  } while (0)

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr uint32_t M_RUN = 1u << ST_RUN;
constexpr uint32_t M_HALF = 1u << ST_HALF;
constexpr uint32_t M_CHECK = 1u << ST_CHECK;
constexpr uint32_t M_INIT = 1u << ST_INIT;
// Finished slots whose last x-forward may not be that of f . x (see farfield_after_solve).
constexpr uint32_t M_STOPPED = (1u << ST_BREAK) | (1u << ST_NONFIN);
constexpr uint32_t M_ALL = (1u << ST_RUN) | (1u << ST_HALF) | (1u << ST_CHECK) | (1u << ST_OK) | (1u << ST_MAXIT) |
                           (1u << ST_BREAK) | (1u << ST_NONFIN) | (1u << ST_INIT);

// Vectors per slot (each N complex) for each operation; the x-spectrum takes two.
int vecs_per_slot(int op) {
  switch (op) {
    case LS_OP_FORWARD: return 12;  // r rh p v s t + spectra (3 x 2)
    case LS_OP_FARFIELD: return 3;  // spectrum(2) + detector x-spectrum
    case LS_OP_GRAD: return 15;     // u wbar b r rh p v s t + spectra (3 x 2)
    default: return 6;              // spectra (3 x 2)
  }
}

struct WsLayout {
  size_t off_desc[3], off_st, off_part, off_stats, off_det, off_grad, off_vec, per_slot, total;
};

WsLayout ws_layout(const ls_ctx* c, int Q, int op) {
  WsLayout L;
  const int nblk = blocks_per_slot(c->n, c->n);
  size_t o = 0;
  for (int i = 0; i < 3; ++i) {
    L.off_desc[i] = o;
    o += al(sizeof(SlotDesc) * (size_t)Q);
  }
  L.off_st = o;
  o += al(sizeof(SlotState) * (size_t)Q);
  L.off_part = o;
  o += al((size_t)Q * nblk * PART_K * 2 * sizeof(double));
  L.off_stats = o;
  o += al((size_t)Q * 2 * sizeof(double));
  L.off_det = o;
  if (op == LS_OP_GRAD) o += al((size_t)Q * c->n * c->n * c->csz);
  L.off_grad = o;
  if (op == LS_OP_GRAD) o += al(c->N * sizeof(double));
  L.off_vec = o;
  L.per_slot = (size_t)vecs_per_slot(op) * c->N * c->csz;
  o += (size_t)Q * L.per_slot;
  L.total = o;
  return L;
}

int fit_slots(const ls_ctx* c, int Q, int op, size_t ws_bytes) {
  int lo = 0, hi = Q;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (ws_layout(c, mid, op).total <= ws_bytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// A group of slots resident on the device.
struct Run {
  const ls_ctx* c;
  hipStream_t s;
  int nslots;
  bool warm = false;  // x0 = the contents of vec[V_X] (else x0 = b)
  SlotDesc* d_desc;
  SlotState* d_st;
  double* d_part;
  PassArgs base() const {
    PassArgs a;
    std::memset(&a, 0, sizeof(a));
    a.desc = d_desc;
    a.st = d_st;
    a.part = d_part;
    a.part_stride = blocks_per_slot(c->n, c->n);
    a.nslots = nslots;
    a.nz = c->n;
    a.tw = c->tw;
    a.kern = c->kvol;
    a.spec = V_SPEC;
    a.spec2 = -1;
    return a;
  }
};

// k_xinv reads the class-major output of the (y,z) pass, which starts at V_SPE and runs over
// V_SPE and V_SPO (4 N complex per slot); spec2 >= 0 selects that mode.
void xinv_source(const ls_ctx* c, PassArgs& a) {
  (void)c;
  a.spec = V_SPE;
  a.spec2 = V_SPO;
}

int matvec(const Run& r, int pro, int sel, int epi, int esel, int esel2, uint32_t mask) {
  PassArgs a = r.base();
  a.mask = mask;
  a.mode = pro;
  a.sel = sel;
  HIPCHK(launch_xfwd(r.c->dbl, r.c->n, a, r.s));
  HIPCHK(launch_yz(r.c->dbl, r.c->n, a, r.s));
  a.mode = epi;
  a.sel = esel;
  a.sel2 = esel2;
  xinv_source(r.c, a);
  HIPCHK(launch_xinv(r.c->dbl, r.c->n, a, r.s));
  return LS_OK;
}

int scalar(const Run& r, int kind, uint32_t mask) {
  PassArgs a = r.base();
  a.mask = mask;
  HIPCHK(launch_scalar(kind, r.c->dbl, a, r.s));
  return LS_OK;
}

// Enqueue: initial residuals of admitted slots, then `iters` BiCGSTAB iterations, then the
// true-residual check of the slots whose recursion finished during them.  Slots not in the state
// a kernel acts on return immediately, so this needs no host round trip; a slot that finishes its
// recursion before the last of the iterations waits (untouched) for the check, so each slot runs
// the same operations in the same order as with a check after every iteration.  Only the host
// admits slots, so it knows whether any is waiting for its initial residual (`init`); if none is,
// those launches are skipped.
int enqueue_steps(const Run& r, int iters, bool init) {
  int rc;
  if (init) {
    if (r.warm) {
      if ((rc = matvec(r, PRO_F_VEC, V_X, EPI_R0X, 0, 0, M_INIT))) return rc;
    } else {
      if ((rc = matvec(r, PRO_F_B, 0, EPI_R0, 0, 0, M_INIT))) return rc;
    }
    if ((rc = scalar(r, SC_INIT, M_INIT))) return rc;
  }
  for (int it = 0; it < iters; ++it) {
    if ((rc = matvec(r, PRO_P, 0, EPI_AXV, 0, 0, M_RUN))) return rc;
    if ((rc = scalar(r, SC_ALPHA, M_RUN))) return rc;
    if ((rc = matvec(r, PRO_S, 0, EPI_AXT, 0, 0, M_RUN))) return rc;
    if ((rc = scalar(r, SC_OMEGA, M_RUN))) return rc;
    {
      PassArgs a = r.base();
      a.mask = M_RUN | M_HALF;
      HIPCHK(launch_update(r.c->dbl, r.c->n, a, r.s));
    }
    if ((rc = scalar(r, SC_BETA, M_RUN | M_HALF))) return rc;
  }
  if (iters > 0) {
    if ((rc = matvec(r, PRO_F_VEC, V_X, EPI_TRUE, 0, 0, M_CHECK))) return rc;
    if ((rc = scalar(r, SC_FINAL, M_CHECK))) return rc;
  }
  return LS_OK;
}

int pull_states(const Run& r, std::vector<SlotState>& h) {
  h.resize(r.nslots);
  HIPCHK(hipMemcpyAsync(h.data(), r.d_st, sizeof(SlotState) * r.nslots, hipMemcpyDeviceToHost, r.s));
  HIPCHK(hipStreamSynchronize(r.s));
  return LS_OK;
}

bool busy(const SlotState& s) {
  return s.status == ST_RUN || s.status == ST_HALF || s.status == ST_CHECK || s.status == ST_INIT;
}

bool any_init(const std::vector<SlotState>& h) {
  for (const auto& s : h)
    if (s.status == ST_INIT) return true;
  return false;
}

int solve_all(const Run& r, std::vector<SlotState>& h) {
  int rc;
  int chunk = 2;
  for (int guard = 0; guard < 100000; ++guard) {
    if ((rc = enqueue_steps(r, chunk, guard == 0 || any_init(h)))) return rc;
    if ((rc = pull_states(r, h))) return rc;
    bool any = false;
    for (const auto& s : h) any = any || busy(s);
    if (!any) return LS_OK;
    chunk = 2;
  }
  g_last_error = "solver loop guard";
  return LS_ERR_HIP;
}

void to_info(const SlotState& s, double clk_khz, ls_solve_info* o) {
  int st = 1;
  switch (s.status) {
    case ST_OK: st = 0; break;
    case ST_MAXIT: st = 1; break;
    case ST_BREAK: st = 2; break;
    case ST_NONFIN: st = 3; break;
    default: st = 1;
  }
  o->status = st;
  o->iters = s.iters;
  o->matvecs = s.matvecs;
  o->restarts = s.restarts;
  o->relres_rec = s.relres;
  o->relres_true = s.relres_true;
  o->time_ms = (s.t_done > s.t_start && s.t_start > 0 && clk_khz > 0) ? (double)(s.t_done - s.t_start) / clk_khz : -1.0;
}

// Breakdown threshold of a solve: the caller's, or the unit roundoff of the field precision.
double breakdown_of(const ls_solve_opts& o, bool dbl) {
  if (o.breakdown > 0.0) return o.breakdown;
  return dbl ? 2.220446049250313e-16 : 1.1920928955078125e-07;
}

SlotState init_state(const ls_solve_opts* o, int status, bool dbl) {
  SlotState s;
  std::memset(&s, 0, sizeof(s));
  s.tol = o->tol;
  s.brk = breakdown_of(*o, dbl);
  s.maxit = o->maxit;
  s.max_restarts = o->max_restarts;
  s.status = status;
  return s;
}

SlotState run_state() {
  ls_solve_opts o;
  o.tol = 1e-5;
  o.maxit = 1;
  o.max_restarts = 0;
  o.x0_mode = 0;
  o.reserved = 0;
  o.breakdown = 0.0;
  return init_state(&o, ST_RUN, false);
}

ls_solve_opts opts_or_default(const ls_solve_opts* o) {
  ls_solve_opts d;
  d.tol = 1e-5;
  d.maxit = 500;
  d.max_restarts = 3;
  d.x0_mode = 0;
  d.reserved = 0;
  d.breakdown = 0.0;
  if (o) d = *o;
  return d;
}

bool opts_ok(const ls_solve_opts& o) {
  return o.tol > 0.0 && std::isfinite(o.tol) && o.maxit >= 1 && o.max_restarts >= 0 && (o.x0_mode == 0 || o.x0_mode == 1) &&
         o.breakdown >= 0.0 && o.breakdown < 1.0;
}

char* vptr(const ls_ctx* c, char* ws, const WsLayout& L, int slot, int k) {
  return ws + L.off_vec + (size_t)slot * L.per_slot + (size_t)k * c->N * c->csz;
}

int upload(const Run& r, const std::vector<SlotDesc>& d, const std::vector<SlotState>* st) {
  HIPCHK(hipMemcpyWithStream(r.d_desc, d.data(), sizeof(SlotDesc) * d.size(), hipMemcpyHostToDevice, r.s));
  if (st) HIPCHK(hipMemcpyWithStream(r.d_st, st->data(), sizeof(SlotState) * st->size(), hipMemcpyHostToDevice, r.s));
  return LS_OK;
}

Run make_run(const ls_ctx* c, char* ws, const WsLayout& L, int nslots, int which_desc, hipStream_t s) {
  Run r;
  r.c = c;
  r.s = s;
  r.nslots = nslots;
  r.d_desc = (SlotDesc*)(ws + L.off_desc[which_desc]);
  r.d_st = (SlotState*)(ws + L.off_st);
  r.d_part = (double*)(ws + L.off_part);
  return r;
}

SlotDesc blank_desc(const ls_ctx* c, const void* f) {
  SlotDesc d;
  std::memset(&d, 0, sizeof(d));
  d.f = f;
  d.k = c->g.kbh;
  return d;
}

// Solver-vector slots of a descriptor: r rh p v s t and the spectrum start at vector k0.
void bind_solver(const ls_ctx* c, char* ws, const WsLayout& L, int slot, int k0, SlotDesc& d) {
  d.vec[V_R] = vptr(c, ws, L, slot, k0 + 0);
  d.vec[V_RH] = vptr(c, ws, L, slot, k0 + 1);
  d.vec[V_P] = vptr(c, ws, L, slot, k0 + 2);
  d.vec[V_V] = vptr(c, ws, L, slot, k0 + 3);
  d.vec[V_S] = vptr(c, ws, L, slot, k0 + 4);
  d.vec[V_T] = vptr(c, ws, L, slot, k0 + 5);
  d.vec[V_SPEC] = vptr(c, ws, L, slot, k0 + 6);
  d.vec[V_SPE] = vptr(c, ws, L, slot, k0 + 8);
  d.vec[V_SPO] = vptr(c, ws, L, slot, k0 + 10);
}

int check_ctx(const ls_ctx* c) { return c && c->kbuf ? LS_OK : LS_ERR_ARG; }

// far field of slot vectors: spectrum of f.vec[sel] -> k_ff -> detector vec[out_sel].  The
// x-forward runs on the slots in xfwd_mask only (the others already hold that spectrum in V_SPEC).
int farfield_run(const Run& r, int sel, int tmp_sel, int out_sel, uint32_t mask, uint32_t xfwd_mask) {
  PassArgs a = r.base();
  a.mask = xfwd_mask;
  a.mode = PRO_F_VEC;
  a.sel = sel;
  a.spec = V_SPEC;
  if (xfwd_mask) HIPCHK(launch_xfwd(r.c->dbl, r.c->n, a, r.s));
  a.mask = mask;
  a.kern = r.c->kff;
  a.spec = V_SPEC;
  a.sel = tmp_sel;
  HIPCHK(launch_ff(r.c->dbl, r.c->n, a, r.s));
  a.mode = EPI_STORE;
  a.sel = out_sel;
  a.spec = tmp_sel;
  a.nz = 1;
  HIPCHK(launch_xinv(r.c->dbl, r.c->n, a, r.s));
  return LS_OK;
}

// out = G~^T (conj?) vec[in_sel] (detector) -> volume vec[out_sel]
int farfield_adj_run(const Run& r, int in_sel, int tmp_sel, int out_sel, bool conj, uint32_t mask) {
  PassArgs a = r.base();
  a.mask = mask;
  a.mode = conj ? PRO_CONJ_VEC : PRO_VEC;
  a.sel = in_sel;
  a.spec = tmp_sel;
  a.nz = 1;
  HIPCHK(launch_xfwd(r.c->dbl, r.c->n, a, r.s));
  a.nz = r.c->n;
  a.kern = r.c->kff;
  a.sel = tmp_sel;
  a.spec = V_SPEC;
  HIPCHK(launch_ffT(r.c->dbl, r.c->n, a, r.s));
  a.mode = EPI_STORE;
  a.sel = out_sel;
  a.spec = V_SPEC;
  HIPCHK(launch_xinv(r.c->dbl, r.c->n, a, r.s));
  return LS_OK;
}

// Far field of the solutions of a finished solve into vec[out_sel].  A slot that ended through the
// initial residual test or the final true-residual check last ran the x-forward of f . x, so its
// V_SPEC already holds the x-spectrum the far field starts from (the same kernel on the same input
// as a separate x-forward: bit for bit the same spectrum); slots that stopped inside the recursion
// (breakdown, non-finite values), or all slots when some x was overwritten after the solve
// (`recompute`), get it recomputed.  V_T (free once the solve is done) holds the detector spectra.
int farfield_after_solve(const Run& r, int out_sel, bool recompute) {
  return farfield_run(r, V_X, V_T, out_sel, M_ALL, recompute ? M_ALL : M_STOPPED);
}

}  // namespace

// =============================================================================================
extern "C" {

const char* ls_strerror(int code) {
  switch (code) {
    case LS_OK: return "ok";
    case LS_ERR_ARG: return "invalid argument";
    case LS_ERR_WORKSPACE: return "workspace or kernel buffer too small";
    case LS_ERR_UNSUPPORTED: return "grid size / precision not supported";
    case LS_ERR_HIP: return "HIP runtime error";
    default: return "unknown error";
  }
}

const char* ls_last_error(void) { return g_last_error.c_str(); }

static int geom_check(const ls_geom* g) {
  if (!g) return LS_ERR_ARG;
  if (g->prec != LS_C64 && g->prec != LS_C128) return LS_ERR_ARG;
  if (g->n < 8 || (g->n % 2)) return LS_ERR_ARG;
  if (g->p < 2 || (g->p % 2)) return LS_ERR_ARG;
  if (!(g->kbh > 0.0 && g->kbh < M_PI)) return LS_ERR_ARG;
  if (!(g->xg > 0.5 * g->n) || !std::isfinite(g->xg)) return LS_ERR_ARG;
  if (!fused_supported(g->n, g->prec == LS_C128)) return LS_ERR_UNSUPPORTED;
  return LS_OK;
}

int ls_kernel_bytes(const ls_geom* g, size_t* bytes) {
  int rc = geom_check(g);
  if (rc) return rc;
  if (!bytes) return LS_ERR_ARG;
  *bytes = kernel_layout(g->n, g->prec == LS_C128).total;
  return LS_OK;
}

int ls_init_workspace_bytes(const ls_geom* g, size_t* bytes) {
  int rc = geom_check(g);
  if (rc) return rc;
  if (!bytes) return LS_ERR_ARG;
  *bytes = init_ws_bytes(g->n);
  return LS_OK;
}

// Fixed device scratch of ls_forward_farfield_noalloc: one copy per device, loaded with the library's
// code object and held until the process ends.  In host code `scratch` names a host-side stand-in,
// not the device array: its device address comes from hipGetSymbolAddress, resolved once per device
// with that device current (scratch_address) and used everywhere host code needs the array.
static __device__ __align__(256) char scratch[LS_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device (resolved on first use per device).
int scratch_address(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    g_last_error = "scratch: device ordinal out of range";
    return LS_ERR_ARG;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) {
      g_last_error = "hipGetSymbolAddress(scratch) returned a null address";
      return LS_ERR_HIP;
    }
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return LS_OK;
}
}  // namespace

int ls_green_init(const ls_geom* g, void* kbuf, size_t kbuf_bytes, void* ws, size_t ws_bytes, void* stream,
                  ls_ctx** out) {
  int rc = geom_check(g);
  if (rc) return rc;
  if (!kbuf || !ws || !out) return LS_ERR_ARG;
  const bool dbl = g->prec == LS_C128;
  const KernelLayout KL = kernel_layout(g->n, dbl);
  if (kbuf_bytes < KL.total || ws_bytes < init_ws_bytes(g->n)) return LS_ERR_WORKSPACE;
  hipError_t e = green_build(g->n, g->p, g->kbh, g->xg, dbl, kbuf, ws, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "green_build");
  int dev = 0, clk = 0;
  HIPCHK(hipGetDevice(&dev));
  if (hipDeviceGetAttribute(&clk, hipDeviceAttributeWallClockRate, dev) != hipSuccess) clk = 0;
  {  // set-up of the fixed scratch on this device (the no-allocation entry point retries if this fails)
    void* p = nullptr;
    (void)scratch_address(&p);
  }
  ls_ctx* c = new (std::nothrow) ls_ctx;
  if (!c) return LS_ERR_ARG;
  c->g = *g;
  c->dbl = dbl;
  c->n = g->n;
  c->csz = dbl ? 16 : 8;
  c->N = (size_t)g->n * g->n * g->n;
  c->kbuf = (char*)kbuf;
  c->tw = c->kbuf + KL.off_tw;
  c->kvol = c->kbuf + KL.off_vol;
  c->kff = c->kbuf + KL.off_ff;
  c->clk_khz = (double)clk;
  *out = c;
  return LS_OK;
}

void ls_ctx_destroy(ls_ctx* ctx) { delete ctx; }

// Reconstruction-step workspace: z, x_r (N reals each), p, r (3 N reals each), TV partial sums.
struct ProxLayout {
  size_t z, xr, p, r, part, total;
};
static ProxLayout prox_layout(const ls_ctx* c) {
  const size_t rsz = c->dbl ? 8 : 4;
  ProxLayout L;
  size_t o = 0;
  L.z = o;
  o += al(c->N * rsz);
  L.xr = o;
  o += al(c->N * rsz);
  L.p = o;
  o += al(3 * c->N * rsz);
  L.r = o;
  o += al(3 * c->N * rsz);
  L.part = o;
  o += al(((size_t)tv_partial_blocks(c->N) + 1) * sizeof(double));
  L.total = o;
  return L;
}

// Incident-field workspace for Q illuminations: FP64 twiddles (n), tilts (2 Q), detector
// spectra (Q n^2) and propagated slices (Q n^3).
struct IncLayout {
  size_t tw, kt, A, B, total;
};
static IncLayout inc_layout(const ls_ctx* c, int Q) {
  IncLayout L;
  const size_t n = c->n, cz = 2 * sizeof(double);
  size_t o = 0;
  L.tw = o;
  o += al(n * cz);
  L.kt = o;
  o += al(2 * (size_t)Q * sizeof(double));
  L.A = o;
  o += al((size_t)Q * n * n * cz);
  L.B = o;
  o += al((size_t)Q * n * n * n * cz);
  L.total = o;
  return L;
}

int ls_workspace_bytes(const ls_ctx* ctx, int32_t Q, int32_t op, size_t* bytes) {
  if (check_ctx(ctx) || Q < 1 || !bytes || op < 0 || op > LS_OP_INCIDENT) return LS_ERR_ARG;
  if (op == LS_OP_PROX)
    *bytes = prox_layout(ctx).total;
  else if (op == LS_OP_INCIDENT)
    *bytes = inc_layout(ctx, Q).total;
  else
    *bytes = ws_layout(ctx, Q, op).total;
  return LS_OK;
}

int ls_incident_field(const ls_ctx* c, const void* y_in, const double* ktilde, int32_t Q, int32_t tilt, void* uin,
                      void* ws, size_t ws_bytes, void* stream) {
  if (check_ctx(c) || !y_in || !uin || !ws || Q < 1 || (tilt && !ktilde)) return LS_ERR_ARG;
  if (tilt)
    for (int i = 0; i < 2 * Q; ++i)
      if (!std::isfinite(ktilde[i])) return LS_ERR_ARG;
  int Qg = 0;
  for (int q = Q; q >= 1 && !Qg; q = q > 1 ? q / 2 : 0)
    if (inc_layout(c, q).total <= ws_bytes) Qg = q;
  if (Qg < 1) return LS_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  const int n = c->n;
  std::vector<double> tw;
  twiddles(n, tw);
  const IncLayout L = inc_layout(c, Qg);
  HIPCHK(hipMemcpyWithStream(w + L.tw, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice, s));
  const size_t M = (size_t)n * n;
  for (int q0 = 0; q0 < Q; q0 += Qg) {
    const int nq = std::min(Qg, Q - q0);
    double* kt = (double*)(w + L.kt);
    if (tilt) HIPCHK(hipMemcpyWithStream(kt, ktilde + 2 * q0, 2 * nq * sizeof(double), hipMemcpyHostToDevice, s));
    cplx<double>* A = (cplx<double>*)(w + L.A);
    cplx<double>* B = (cplx<double>*)(w + L.B);
    const cplx<double>* twd = (const cplx<double>*)(w + L.tw);
    HIPCHK(launch_inc_demod(c->dbl, (const char*)y_in + (size_t)q0 * M * c->csz, kt, tilt != 0, A, n, nq, s));
    HIPCHK(fft2_batched(n, -1, A, nq, twd, s));
    HIPCHK(launch_inc_prop(A, kt, tilt != 0, c->g.kbh, c->g.xg, B, n, nq, s));
    HIPCHK(fft2_batched(n, +1, B, nq * n, twd, s));
    HIPCHK(launch_inc_mod(c->dbl, B, kt, tilt != 0, (char*)uin + (size_t)q0 * M * n * c->csz, n, nq, s));
  }
  return LS_OK;
}

int ls_prox_tv(const ls_ctx* c, const void* v, const void* d, double gamma, double lam, int32_t iters,
               int32_t nonneg, void* x, void* ws, size_t ws_bytes, void* stream) {
  if (check_ctx(c) || !v || !x || !ws || iters < 0 || !(lam >= 0.0) || !std::isfinite(lam) || !std::isfinite(gamma))
    return LS_ERR_ARG;
  const ProxLayout L = prox_layout(c);
  if (ws_bytes < L.total) return LS_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  void *z = w + L.z, *xr = w + L.xr, *p = w + L.p, *r = w + L.r;
  HIPCHK(launch_prox_init(c->dbl, v, d, gamma, z, p, r, c->N, s));
  if (lam > 0.0 && iters > 0) {
    double t = 1.0;
    for (int k = 0; k < iters; ++k) {
      HIPCHK(launch_prox_primal(c->dbl, z, r, lam, nonneg != 0, xr, c->n, s));
      const double t_next = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
      HIPCHK(launch_prox_dual(c->dbl, xr, p, r, 1.0 / (12.0 * lam), (t - 1.0) / t_next, c->n, s));
      t = t_next;
    }
  }
  // x = P_C(z - lam D^T p); p = 0 when no dual step ran
  HIPCHK(launch_prox_primal(c->dbl, z, p, lam, nonneg != 0, x, c->n, s));
  return LS_OK;
}

int ls_fbs_extrapolate(const ls_ctx* c, const void* f, const void* f_prev, double beta, void* v_out, void* stream) {
  if (check_ctx(c) || !f || !f_prev || !v_out || !std::isfinite(beta)) return LS_ERR_ARG;
  HIPCHK(launch_extrapolate(c->dbl, f, f_prev, beta, v_out, c->N, (hipStream_t)stream));
  return LS_OK;
}

int ls_tv_value(const ls_ctx* c, const void* x, double* out, void* ws, size_t ws_bytes, void* stream) {
  if (check_ctx(c) || !x || !out || !ws) return LS_ERR_ARG;
  const ProxLayout L = prox_layout(c);
  if (ws_bytes < L.total) return LS_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  double* part = (double*)((char*)ws + L.part);
  const int nb = tv_partial_blocks(c->N);
  HIPCHK(launch_tv_value(c->dbl, x, c->n, part, part + nb, s));
  HIPCHK(hipMemcpyWithStream(out, part + nb, sizeof(double), hipMemcpyDeviceToHost, s));
  return LS_OK;
}

static int apply_common(const ls_ctx* c, const void* f, const void* v, void* out, int32_t Q, void* ws,
                        size_t ws_bytes, void* stream, bool withA) {
  if (check_ctx(c) || !v || !out || !ws || Q < 1 || (withA && !f)) return LS_ERR_ARG;
  const int Qg = fit_slots(c, Q, LS_OP_APPLY, ws_bytes);
  if (Qg < 1) return LS_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  for (int q0 = 0; q0 < Q; q0 += Qg) {
    const int nq = std::min(Qg, Q - q0);
    const WsLayout L = ws_layout(c, nq, LS_OP_APPLY);
    std::vector<SlotDesc> d(nq);
    std::vector<SlotState> st(nq, run_state());
    for (int i = 0; i < nq; ++i) {
      d[i] = blank_desc(c, f);
      d[i].vec[V_X] = (char*)v + (size_t)(q0 + i) * c->N * c->csz;
      d[i].vec[V_R] = (char*)out + (size_t)(q0 + i) * c->N * c->csz;
      d[i].vec[V_SPEC] = vptr(c, w, L, i, 0);
      d[i].vec[V_SPE] = vptr(c, w, L, i, 2);
      d[i].vec[V_SPO] = vptr(c, w, L, i, 4);
    }
    Run r = make_run(c, w, L, nq, 0, s);
    int rc = upload(r, d, &st);
    if (rc) return rc;
    if (withA)
      rc = matvec(r, PRO_F_VEC, V_X, EPI_AX, V_X, V_R, M_RUN);
    else
      rc = matvec(r, PRO_VEC, V_X, EPI_STORE, V_R, 0, M_RUN);
    if (rc) return rc;
  }
  return LS_OK;
}

int ls_apply_G(const ls_ctx* ctx, const void* v, void* out, int32_t Q, void* ws, size_t ws_bytes, void* stream) {
  return apply_common(ctx, nullptr, v, out, Q, ws, ws_bytes, stream, false);
}

int ls_apply_A(const ls_ctx* ctx, const void* f, const void* v, void* out, int32_t Q, void* ws, size_t ws_bytes,
               void* stream) {
  return apply_common(ctx, f, v, out, Q, ws, ws_bytes, stream, true);
}

// Forward solves with plane-wave (dirs) or stored (uin) incident fields; with y, also the far
// field of every solution.
static int forward_common(const ls_ctx* c, const void* f, int32_t Q, const double* dirs, const void* uin, void* u,
                          void* y, const ls_solve_opts* opts, ls_solve_info* info, void* ws, size_t ws_bytes,
                          void* stream) {
  const ls_solve_opts o = opts_or_default(opts);
  if (!opts_ok(o)) return LS_ERR_ARG;
  const int Qg = fit_slots(c, Q, LS_OP_FORWARD, ws_bytes);
  if (Qg < 1) return LS_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  std::vector<SlotState> h;
  for (int q0 = 0; q0 < Q; q0 += Qg) {
    const int nq = std::min(Qg, Q - q0);
    const WsLayout L = ws_layout(c, nq, LS_OP_FORWARD);
    std::vector<SlotDesc> d(nq);
    std::vector<SlotState> st(nq, init_state(&o, ST_INIT, c->dbl));
    for (int i = 0; i < nq; ++i) {
      d[i] = blank_desc(c, f);
      d[i].vec[V_X] = (char*)u + (size_t)(q0 + i) * c->N * c->csz;
      bind_solver(c, w, L, i, 0, d[i]);
      if (y) d[i].vec[V_AUX] = (char*)y + (size_t)(q0 + i) * c->n * c->n * c->csz;
      if (uin)
        d[i].vec[V_B] = (void*)((const char*)uin + (size_t)(q0 + i) * c->N * c->csz);
      else
        for (int j = 0; j < 3; ++j) d[i].d[j] = dirs[3 * (q0 + i) + j];
    }
    Run r = make_run(c, w, L, nq, 0, s);
    r.warm = o.x0_mode == 1;
    int rc = upload(r, d, &st);
    if (rc) return rc;
    if ((rc = solve_all(r, h))) return rc;
    // A zero right-hand side has the solution zero; a warm start would otherwise hand back the
    // caller's guess, since the initial residual test accepts ||b|| = 0 before any update.
    bool zeroed = false;
    if (r.warm)
      for (int i = 0; i < nq; ++i)
        if (h[i].status == ST_OK && h[i].nb == 0.0) {
          HIPCHK(hipMemsetAsync(d[i].vec[V_X], 0, c->N * c->csz, s));
          zeroed = true;
        }
    if (y && (rc = farfield_after_solve(r, V_AUX, zeroed))) return rc;
    if (info)
      for (int i = 0; i < nq; ++i) to_info(h[i], c->clk_khz, info + q0 + i);
  }
  return LS_OK;
}

int ls_forward(const ls_ctx* c, const void* f, int32_t Q, const double* dirs, void* u, const ls_solve_opts* opts,
               ls_solve_info* info, void* ws, size_t ws_bytes, void* stream) {
  if (check_ctx(c) || !f || !dirs || !u || !ws || Q < 1) return LS_ERR_ARG;
  return forward_common(c, f, Q, dirs, nullptr, u, nullptr, opts, info, ws, ws_bytes, stream);
}

int ls_forward_farfield(const ls_ctx* c, const void* f, int32_t Q, const double* dirs, void* u, void* y,
                        const ls_solve_opts* opts, ls_solve_info* info, void* ws, size_t ws_bytes, void* stream) {
  if (check_ctx(c) || !f || !dirs || !u || !y || !ws || Q < 1) return LS_ERR_ARG;
  return forward_common(c, f, Q, dirs, nullptr, u, y, opts, info, ws, ws_bytes, stream);
}

int ls_forward_farfield_noalloc(const ls_ctx* c, const void* f, int32_t Q, const double* dirs, void* u, void* y,
                                const ls_solve_opts* opts, ls_solve_info* info, void* stream) {
  if (check_ctx(c) || !f || !dirs || !u || !y || Q < 1) return LS_ERR_ARG;
  if (ws_layout(c, 1, LS_OP_FORWARD).total > (size_t)LS_SCRATCH_BYTES) {
    g_last_error = "ls_forward_farfield_noalloc: one illumination of this grid needs " +
                   std::to_string(ws_layout(c, 1, LS_OP_FORWARD).total) + " bytes of scratch, more than the " +
                   std::to_string((size_t)LS_SCRATCH_BYTES) + " bytes of the fixed device scratch";
    return LS_ERR_WORKSPACE;
  }
  void* ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc) return rc;
  return forward_common(c, f, Q, dirs, nullptr, u, y, opts, info, ws, (size_t)LS_SCRATCH_BYTES, stream);
}

int ls_forward_uin(const ls_ctx* c, const void* f, int32_t Q, const void* uin, void* u, const ls_solve_opts* opts,
                   ls_solve_info* info, void* ws, size_t ws_bytes, void* stream) {
  if (check_ctx(c) || !f || !uin || !u || !ws || Q < 1 || uin == u) return LS_ERR_ARG;
  return forward_common(c, f, Q, nullptr, uin, u, nullptr, opts, info, ws, ws_bytes, stream);
}

int ls_farfield(const ls_ctx* c, const void* f, const void* u, int32_t Q, void* y, void* ws, size_t ws_bytes,
                void* stream) {
  if (check_ctx(c) || !f || !u || !y || !ws || Q < 1) return LS_ERR_ARG;
  const int Qg = fit_slots(c, Q, LS_OP_FARFIELD, ws_bytes);
  if (Qg < 1) return LS_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  const size_t M = (size_t)c->n * c->n;
  for (int q0 = 0; q0 < Q; q0 += Qg) {
    const int nq = std::min(Qg, Q - q0);
    const WsLayout L = ws_layout(c, nq, LS_OP_FARFIELD);
    std::vector<SlotDesc> d(nq);
    std::vector<SlotState> st(nq, run_state());
    for (int i = 0; i < nq; ++i) {
      d[i] = blank_desc(c, f);
      d[i].vec[V_X] = (char*)u + (size_t)(q0 + i) * c->N * c->csz;
      d[i].vec[V_SPEC] = vptr(c, w, L, i, 0);
      d[i].vec[V_T] = vptr(c, w, L, i, 2);
      d[i].vec[V_AUX] = (char*)y + (size_t)(q0 + i) * M * c->csz;
    }
    Run r = make_run(c, w, L, nq, 0, s);
    int rc = upload(r, d, &st);
    if (rc) return rc;
    if ((rc = farfield_run(r, V_X, V_T, V_AUX, M_RUN, M_RUN))) return rc;
  }
  return LS_OK;
}

int ls_farfield_adj(const ls_ctx* c, const void* rdet, int32_t conj, int32_t Q, void* out, void* ws, size_t ws_bytes,
                    void* stream) {
  if (check_ctx(c) || !rdet || !out || !ws || Q < 1) return LS_ERR_ARG;
  const int Qg = fit_slots(c, Q, LS_OP_FARFIELD, ws_bytes);
  if (Qg < 1) return LS_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  const size_t M = (size_t)c->n * c->n;
  for (int q0 = 0; q0 < Q; q0 += Qg) {
    const int nq = std::min(Qg, Q - q0);
    const WsLayout L = ws_layout(c, nq, LS_OP_FARFIELD);
    std::vector<SlotDesc> d(nq);
    std::vector<SlotState> st(nq, run_state());
    for (int i = 0; i < nq; ++i) {
      d[i] = blank_desc(c, nullptr);
      d[i].vec[V_AUX] = (char*)rdet + (size_t)(q0 + i) * M * c->csz;
      d[i].vec[V_SPEC] = vptr(c, w, L, i, 0);
      d[i].vec[V_T] = vptr(c, w, L, i, 2);
      d[i].vec[V_B] = (char*)out + (size_t)(q0 + i) * c->N * c->csz;
    }
    Run r = make_run(c, w, L, nq, 0, s);
    int rc = upload(r, d, &st);
    if (rc) return rc;
    if ((rc = farfield_adj_run(r, V_AUX, V_T, V_B, conj != 0, M_RUN))) return rc;
  }
  return LS_OK;
}

// Shared driver of ls_vjp and ls_grad.
static int grad_driver(const ls_ctx* c, const void* f, int32_t Q, const double* dirs, const void* u_in,
                       const void* gy, const void* y_meas, const void* rhs, void* grad, double* loss,
                       const ls_solve_opts* opts, ls_solve_info* info, void* ws, size_t ws_bytes, void* stream) {
  const ls_solve_opts o = opts_or_default(opts);
  if (!opts_ok(o)) return LS_ERR_ARG;
  const int Qg = fit_slots(c, Q, LS_OP_GRAD, ws_bytes);
  if (Qg < 1) return LS_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  const size_t M = (size_t)c->n * c->n;
  const bool full = (y_meas != nullptr);
  double loss_acc = 0.0;
  std::vector<SlotState> h;
  double* d_grad = nullptr;
  for (int q0 = 0; q0 < Q; q0 += Qg) {
    const int nq = std::min(Qg, Q - q0);
    const WsLayout L = ws_layout(c, nq, LS_OP_GRAD);
    d_grad = (double*)(w + L.off_grad);
    double* d_stats = (double*)(w + L.off_stats);
    char* det = w + L.off_det;
    int rc;
    // vectors: 0 u, 1 wbar, 2 b, 3.. solver
    std::vector<SlotDesc> dfw(nq), dad(nq), dgr(nq);
    for (int i = 0; i < nq; ++i) {
      const void* uq = full ? (const void*)vptr(c, w, L, i, 0) : (const void*)((const char*)u_in + (size_t)(q0 + i) * c->N * c->csz);
      dfw[i] = blank_desc(c, f);
      dfw[i].vec[V_X] = (void*)uq;
      bind_solver(c, w, L, i, 3, dfw[i]);
      if (dirs)
        for (int j = 0; j < 3; ++j) dfw[i].d[j] = dirs[3 * (q0 + i) + j];
      dfw[i].vec[V_AUX] = det + (size_t)i * M * c->csz;
      dad[i] = blank_desc(c, f);
      dad[i].vec[V_X] = vptr(c, w, L, i, 1);
      dad[i].vec[V_B] = rhs ? (void*)((const char*)rhs + (size_t)(q0 + i) * c->N * c->csz) : vptr(c, w, L, i, 2);
      bind_solver(c, w, L, i, 3, dad[i]);
      dad[i].vec[V_AUX] = full ? (void*)(det + (size_t)i * M * c->csz)
                               : (void*)((const char*)gy + (size_t)(q0 + i) * M * c->csz);
      dgr[i] = blank_desc(c, f);
      dgr[i].vec[V_X] = (void*)uq;
      dgr[i].vec[V_R] = vptr(c, w, L, i, 1);
    }
    Run rf = make_run(c, w, L, nq, 0, s);
    Run ra = make_run(c, w, L, nq, 1, s);
    std::vector<SlotState> st(nq, init_state(&o, ST_INIT, c->dbl));
    if ((rc = upload(rf, dfw, &st))) return rc;
    if ((rc = upload(ra, dad, nullptr))) return rc;
    HIPCHK(hipMemcpyWithStream(w + L.off_desc[2], dgr.data(), sizeof(SlotDesc) * nq, hipMemcpyHostToDevice, s));
    if (full) {
      if ((rc = solve_all(rf, h))) return rc;
      if (info)
        for (int i = 0; i < nq; ++i) to_info(h[i], c->clk_khz, info + q0 + i);
      // y = G~(f . u) into the detector buffer, then r = y - y_meas in place with FP64 norms
      if ((rc = farfield_after_solve(rf, V_AUX, false))) return rc;
      HIPCHK(launch_residual(c->dbl, c->n, det, (const char*)y_meas + (size_t)q0 * M * c->csz, nq, false, det,
                             d_stats, nullptr, s));
      std::vector<double> hs(2 * nq);
      HIPCHK(hipMemcpyAsync(hs.data(), d_stats, sizeof(double) * 2 * nq, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int i = 0; i < nq; ++i) loss_acc += hs[2 * i] / (2.0 * hs[2 * i + 1]);
      if ((rc = upload(ra, dad, &st))) return rc;
    }
    // b = G~^T conj(r) (unless given): slots are in ST_INIT, the passes act on them without changing state
    if (!rhs && (rc = farfield_adj_run(ra, V_AUX, V_T, V_B, true, M_INIT))) return rc;
    if ((rc = solve_all(ra, h))) return rc;
    if (info) {
      ls_solve_info* base = full ? info + Q : info;
      for (int i = 0; i < nq; ++i) to_info(h[i], c->clk_khz, base + q0 + i);
    }
    HIPCHK(launch_grad_accum(c->dbl, c->n, (const SlotDesc*)(w + L.off_desc[2]), full ? d_stats : nullptr, nq, V_X,
                             V_R, d_grad, q0 > 0 ? 1 : 0, s));
  }
  HIPCHK(launch_convert(c->dbl, d_grad, grad, c->N, s));
  HIPCHK(hipStreamSynchronize(s));
  if (loss) *loss = loss_acc;
  return LS_OK;
}

int ls_vjp(const ls_ctx* c, const void* f, const void* u, int32_t Q, const void* gy, void* grad,
           const ls_solve_opts* opts, ls_solve_info* info, void* ws, size_t ws_bytes, void* stream) {
  if (check_ctx(c) || !f || !u || !gy || !grad || !ws || Q < 1) return LS_ERR_ARG;
  return grad_driver(c, f, Q, nullptr, u, gy, nullptr, nullptr, grad, nullptr, opts, info, ws, ws_bytes, stream);
}

int ls_vjp_rhs(const ls_ctx* c, const void* f, const void* u, int32_t Q, const void* b, void* grad,
               const ls_solve_opts* opts, ls_solve_info* info, void* ws, size_t ws_bytes, void* stream) {
  if (check_ctx(c) || !f || !u || !b || !grad || !ws || Q < 1) return LS_ERR_ARG;
  return grad_driver(c, f, Q, nullptr, u, nullptr, nullptr, b, grad, nullptr, opts, info, ws, ws_bytes, stream);
}

int ls_grad(const ls_ctx* c, const void* f, int32_t Q, const double* dirs, const void* y_meas, void* grad,
            double* loss, const ls_solve_opts* opts, ls_solve_info* info, void* ws, size_t ws_bytes, void* stream) {
  if (check_ctx(c) || !f || !dirs || !y_meas || !grad || !ws || Q < 1) return LS_ERR_ARG;
  return grad_driver(c, f, Q, dirs, nullptr, nullptr, y_meas, nullptr, grad, loss, opts, info, ws, ws_bytes, stream);
}

// ---- detector-side operators
static int det_fft_size(int need) {
  static const int sizes[] = {8, 16, 32, 64, 96, 128, 144, 192, 256, 288, 384, 512};
  for (int v : sizes)
    if (v >= need) return v;
  return 0;
}
static const int kDetSizes[] = {8, 16, 32, 64, 96, 128, 144, 192, 256, 288, 384, 512};
static bool det_size_ok(int M) {
  for (int v : kDetSizes)
    if (v == M) return true;
  return false;
}

// wide far field / its transpose: tw (M), K^ (n M^2), V (n M^2), Y (M^2); pupil: tw (2m), planes
struct DetLayout {
  size_t tw, K, V, Y, total;
};
static DetLayout det_layout(const ls_ctx* c, int M) {
  DetLayout L;
  const size_t cz = 2 * sizeof(double), MM = (size_t)M * M;
  size_t o = 0;
  L.tw = o;
  o += al((size_t)M * cz);
  L.K = o;
  o += al((size_t)c->n * MM * cz);
  L.V = o;
  o += al((size_t)c->n * MM * cz);
  L.Y = o;
  o += al(MM * cz);
  L.total = o;
  return L;
}

static hipError_t upload_twiddles(int M, void* dst, hipStream_t s) {
  std::vector<double> tw;
  twiddles(M, tw);
  return hipMemcpyWithStream(dst, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice, s);
}

int ls_detector_bytes(const ls_ctx* c, int32_t m, size_t* bytes) {
  if (check_ctx(c) || !bytes || m < 1) return LS_ERR_ARG;
  size_t b = 0;
  if (m >= c->n && (m - c->n) % 2 == 0) {
    const int M = det_fft_size(m + c->n - 1);
    if (M) b = det_layout(c, M).total;
  }
  const size_t pb = al(2 * (size_t)m * 2 * sizeof(double)) + al(4 * (size_t)m * m * 2 * sizeof(double));
  *bytes = std::max(b, pb);
  return LS_OK;
}

static int wide_check(const ls_ctx* c, int m, int& M) {
  if (m < c->n || (m - c->n) % 2) return LS_ERR_ARG;
  M = det_fft_size(m + c->n - 1);
  return M ? LS_OK : LS_ERR_UNSUPPORTED;
}

int ls_farfield_wide(const ls_ctx* c, int32_t m, const void* f, const void* u, int32_t Q, void* y, void* ws,
                     size_t ws_bytes, void* stream) {
  if (check_ctx(c) || !f || !u || !y || !ws || Q < 1) return LS_ERR_ARG;
  int M, rc;
  if ((rc = wide_check(c, m, M))) return rc;
  const DetLayout L = det_layout(c, M);
  if (ws_bytes < L.total) return LS_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  cplx<double>* tw = (cplx<double>*)(w + L.tw);
  HIPCHK(upload_twiddles(M, tw, s));
  HIPCHK(launch_det_kernel(w + L.K, c->n, M, (m - c->n) / 2, c->g.kbh, c->g.xg, s));
  HIPCHK(fft2_batched(M, -1, (cplx<double>*)(w + L.K), c->n, tw, s));
  const size_t mm = (size_t)m * m;
  for (int q = 0; q < Q; ++q) {
    HIPCHK(launch_det_pad_vol(c->dbl, f, (const char*)u + (size_t)q * c->N * c->csz, w + L.V, c->n, M, s));
    HIPCHK(fft2_batched(M, -1, (cplx<double>*)(w + L.V), c->n, tw, s));
    HIPCHK(launch_det_mulsum(w + L.K, w + L.V, w + L.Y, c->n, M, s));
    HIPCHK(fft2_batched(M, +1, (cplx<double>*)(w + L.Y), 1, tw, s));
    HIPCHK(launch_det_crop(c->dbl, w + L.Y, (char*)y + (size_t)q * mm * c->csz, m, M, 1, 1.0 / ((double)M * M), s));
  }
  return LS_OK;
}

int ls_farfield_wide_adj(const ls_ctx* c, int32_t m, const void* r, int32_t conj, int32_t Q, void* out, void* ws,
                         size_t ws_bytes, void* stream) {
  if (check_ctx(c) || !r || !out || !ws || Q < 1) return LS_ERR_ARG;
  int M, rc;
  if ((rc = wide_check(c, m, M))) return rc;
  const DetLayout L = det_layout(c, M);
  if (ws_bytes < L.total) return LS_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  cplx<double>* tw = (cplx<double>*)(w + L.tw);
  HIPCHK(upload_twiddles(M, tw, s));
  HIPCHK(launch_det_kernel(w + L.K, c->n, M, (m - c->n) / 2, c->g.kbh, c->g.xg, s));
  HIPCHK(fft2_batched(M, -1, (cplx<double>*)(w + L.K), c->n, tw, s));
  const size_t mm = (size_t)m * m;
  for (int q = 0; q < Q; ++q) {
    HIPCHK(launch_det_pad2(c->dbl, (const char*)r + (size_t)q * mm * c->csz, w + L.Y, m, M, 1, conj != 0, s));
    HIPCHK(fft2_batched(M, -1, (cplx<double>*)(w + L.Y), 1, tw, s));
    HIPCHK(launch_det_mulT(w + L.K, w + L.Y, w + L.V, c->n, M, s));
    HIPCHK(fft2_batched(M, +1, (cplx<double>*)(w + L.V), c->n, tw, s));
    HIPCHK(launch_det_crop(c->dbl, w + L.V, (char*)out + (size_t)q * c->N * c->csz, c->n, M, c->n,
                           1.0 / ((double)M * M), s));
  }
  return LS_OK;
}

int ls_pupil(const ls_ctx* c, int32_t m, const void* y, int32_t Q, double na, double dz, int32_t adjoint, void* out,
             void* ws, size_t ws_bytes, void* stream) {
  if (check_ctx(c) || !y || !out || !ws || Q < 1 || m < 1 || !(na >= 0.0) || !std::isfinite(na) || !std::isfinite(dz))
    return LS_ERR_ARG;
  const int M = 2 * m;
  if (!det_size_ok(M)) return LS_ERR_UNSUPPORTED;
  const size_t cz = 2 * sizeof(double), plane = (size_t)M * M * cz;
  const size_t head = al((size_t)M * cz);
  if (ws_bytes < head + plane) return LS_ERR_WORKSPACE;
  const int Qg = (int)std::min<size_t>((size_t)Q, (ws_bytes - head) / plane);
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  cplx<double>* tw = (cplx<double>*)w;
  HIPCHK(upload_twiddles(M, tw, s));
  const size_t mm = (size_t)m * m;
  for (int q0 = 0; q0 < Q; q0 += Qg) {
    const int nq = std::min(Qg, Q - q0);
    cplx<double>* P = (cplx<double>*)(w + head);
    HIPCHK(launch_det_pad2(c->dbl, (const char*)y + (size_t)q0 * mm * c->csz, P, m, M, nq, 0, s));
    HIPCHK(fft2_batched(M, -1, P, nq, tw, s));
    HIPCHK(launch_det_pupil(P, M, nq, c->g.kbh, na * c->g.kbh, dz, adjoint != 0, s));
    HIPCHK(fft2_batched(M, +1, P, nq, tw, s));
    HIPCHK(launch_det_crop(c->dbl, P, (char*)out + (size_t)q0 * mm * c->csz, m, M, nq, 1.0 / ((double)M * M), s));
  }
  return LS_OK;
}

int ls_decimate(const ls_ctx* c, int32_t m, int32_t q, const void* y, int32_t Q, void* out, int32_t transpose,
                void* stream) {
  if (check_ctx(c) || !y || !out || Q < 1 || m < 1 || q < 1 || m % q || y == out) return LS_ERR_ARG;
  const int s0 = (m / 2 - 1) % q;
  HIPCHK(launch_decimate(c->dbl, y, out, m, q, s0, Q, transpose != 0, (hipStream_t)stream));
  return LS_OK;
}

int ls_profile_pass(const ls_ctx* c, const void* f, void* u, int32_t pass, int32_t Q, int32_t reps, void* ws,
                    size_t ws_bytes, void* stream) {
  if (check_ctx(c) || !f || !u || !ws || Q < 1 || reps < 0 || pass < 0 || pass > 3) return LS_ERR_ARG;
  const WsLayout L = ws_layout(c, Q, LS_OP_FORWARD);
  if (ws_bytes < L.total) return LS_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  std::vector<SlotDesc> d(Q);
  ls_solve_opts o = opts_or_default(nullptr);
  SlotState st0 = init_state(&o, ST_RUN, c->dbl);
  st0.alpha[0] = st0.omega[0] = st0.beta[0] = 0.5;
  std::vector<SlotState> st(Q, st0);
  for (int i = 0; i < Q; ++i) {
    d[i] = blank_desc(c, f);
    d[i].vec[V_X] = (char*)u + (size_t)i * c->N * c->csz;
    bind_solver(c, w, L, i, 0, d[i]);
  }
  Run r = make_run(c, w, L, Q, 0, s);
  int rc = upload(r, d, &st);
  if (rc) return rc;
  PassArgs a = r.base();
  a.mask = M_RUN;
  for (int it = 0; it < reps; ++it) {
    if (pass == 0) {
      a.mode = PRO_P;
      HIPCHK(launch_xfwd(c->dbl, c->n, a, s));
    } else if (pass == 1) {
      HIPCHK(launch_yz(c->dbl, c->n, a, s));
    } else if (pass == 2) {
      a.mode = EPI_AXV;
      xinv_source(c, a);
      HIPCHK(launch_xinv(c->dbl, c->n, a, s));
    } else {
      HIPCHK(launch_update(c->dbl, c->n, a, s));
    }
  }
  return LS_OK;
}

int ls_residual(const ls_ctx* c, const void* y, const void* y_meas, int32_t Q, int32_t weighted, void* r,
                double* stats, double* loss, void* stream) {
  if (check_ctx(c) || !y || !y_meas || !r || !stats || Q < 1) return LS_ERR_ARG;
  HIPCHK(launch_residual(c->dbl, c->n, y, y_meas, Q, weighted != 0, r, stats, loss, (hipStream_t)stream));
  return LS_OK;
}

int ls_grad_accumulate(const ls_ctx* c, const void* u, const void* wb, int32_t Q, const double* stats, void* grad,
                       int32_t accumulate, void* stream) {
  if (check_ctx(c) || !u || !wb || !grad || Q < 1) return LS_ERR_ARG;
  HIPCHK(launch_grad_sum(c->dbl, u, wb, Q, c->N, stats, grad, accumulate, (hipStream_t)stream));
  return LS_OK;
}

}  // extern "C"

// =============================================================================================
// slot pool
struct ls_batch {
  const ls_ctx* c;
  int nslots;
  char* ws;
  WsLayout L;
  ls_solve_opts o;
  std::vector<SlotDesc> hd;
  std::vector<SlotState> hs;
};

extern "C" {

int ls_batch_bytes(const ls_ctx* c, int32_t nslots, size_t* bytes) {
  if (check_ctx(c) || nslots < 1 || !bytes) return LS_ERR_ARG;
  *bytes = ws_layout(c, nslots, LS_OP_FORWARD).total;
  return LS_OK;
}

int ls_batch_create(const ls_ctx* c, int32_t nslots, void* ws, size_t ws_bytes, const ls_solve_opts* opts,
                    ls_batch** out) {
  if (check_ctx(c) || nslots < 1 || !ws || !out) return LS_ERR_ARG;
  const ls_solve_opts o = opts_or_default(opts);
  if (!opts_ok(o)) return LS_ERR_ARG;
  const WsLayout L = ws_layout(c, nslots, LS_OP_FORWARD);
  if (ws_bytes < L.total) return LS_ERR_WORKSPACE;
  ls_batch* b = new (std::nothrow) ls_batch;
  if (!b) return LS_ERR_ARG;
  b->c = c;
  b->nslots = nslots;
  b->ws = (char*)ws;
  b->L = L;
  b->o = o;
  b->hd.assign(nslots, blank_desc(c, nullptr));
  b->hs.assign(nslots, init_state(&o, ST_IDLE, c->dbl));
  for (int i = 0; i < nslots; ++i) bind_solver(c, b->ws, L, i, 0, b->hd[i]);
  Run r = make_run(c, b->ws, L, nslots, 0, nullptr);
  int rc = upload(r, b->hd, &b->hs);
  if (rc) {
    delete b;
    return rc;
  }
  HIPCHK(hipStreamSynchronize(nullptr));
  *out = b;
  return LS_OK;
}

int ls_batch_admit(ls_batch* b, int32_t slot, const void* f, const double* dir, const void* rhs, void* x,
                   void* stream) {
  if (!b || slot < 0 || slot >= b->nslots || !f || !x || (!dir && !rhs)) return LS_ERR_ARG;
  if (b->hs[slot].status != ST_IDLE) return LS_ERR_ARG;
  SlotDesc& d = b->hd[slot];
  d.f = f;
  d.vec[V_X] = x;
  d.vec[V_B] = (void*)rhs;
  for (int j = 0; j < 3; ++j) d.d[j] = dir ? dir[j] : 0.0;
  b->hs[slot] = init_state(&b->o, ST_INIT, b->c->dbl);
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipMemcpyWithStream((SlotDesc*)(b->ws + b->L.off_desc[0]) + slot, &d, sizeof(SlotDesc),
                             hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyWithStream((SlotState*)(b->ws + b->L.off_st) + slot, &b->hs[slot], sizeof(SlotState),
                             hipMemcpyHostToDevice, s));
  return LS_OK;
}

int ls_batch_step(ls_batch* b, int32_t iters, void* stream) {
  if (!b || iters < 0) return LS_ERR_ARG;
  Run r = make_run(b->c, b->ws, b->L, b->nslots, 0, (hipStream_t)stream);
  int rc = enqueue_steps(r, iters, any_init(b->hs));
  if (rc) return rc;
  return pull_states(r, b->hs);
}

int ls_batch_poll(const ls_batch* b, int32_t* state, ls_solve_info* info) {
  if (!b) return LS_ERR_ARG;
  for (int i = 0; i < b->nslots; ++i) {
    const SlotState& s = b->hs[i];
    if (state) state[i] = s.status == ST_IDLE ? 0 : (busy(s) ? 1 : 2);
    if (info) to_info(s, b->c->clk_khz, info + i);
  }
  return LS_OK;
}

int ls_batch_release(ls_batch* b, int32_t slot) {
  if (!b || slot < 0 || slot >= b->nslots) return LS_ERR_ARG;
  if (busy(b->hs[slot])) return LS_ERR_ARG;
  b->hs[slot].status = ST_IDLE;
  HIPCHK(hipMemcpy((SlotState*)(b->ws + b->L.off_st) + slot, &b->hs[slot], sizeof(SlotState), hipMemcpyHostToDevice));
  return LS_OK;
}

void ls_batch_destroy(ls_batch* b) { delete b; }

}  // extern "C"
