// Internal context of the magfft library (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/magfft.h"

namespace mag {

// Per-call iteration state kept in device memory.  Kernels of an iteration
// read `done` and return at once when it is set, so a block of iterations can
// be enqueued without host round trips.
struct IterState {
  int done;       // 1 once the stop test passed (or the fixed count is reached)
  int iters;      // inner iterations performed (film: evaluations of (11))
  int fixed;      // fixed iteration count, 0 = stop test
  int fail;       // sticky: set with done = 2; kept by the reset that starts an
                  // evaluation queued behind an unchecked asynchronous one
  int cold;       // the stencil starts the free space from dh_e/dt, not from the warm start
  int pad;
  double thr;     // stop threshold tol * max(|dh_e/dt|, 1)
  double inv_nout;
  double C;       // film: free-space mean of G, eq. (11)
  double A;       // film: pending constant shift of (10)/(12)
  double r;       // last residual
  double sum0;    // scratch
  double hde;     // dh_e/dt of the right-hand side (film: z component), read by
                  // the stencil and the iteration passes
};

// Step control of a device-driven integration (mag_integrate_captured): the
// kernels of a step attempt read t and h here, the accept kernel updates them
// and copies the record to a coherent pinned mirror that the host reads.
struct StepCtl {
  double t, h, t_end, rtol, atol;
  double err;      // error norm of the last attempt
  int accepted;    // attempts accepted since the start of the run
  int rejected;    // attempts rejected
  int commit;      // the last attempt was accepted: y <- y_new, k1 <- k4
  int finished;    // t reached t_end or a status was set: every step kernel returns at once
  int status;      // 0 or MAG_STEP_UNDERFLOW
  int pad;
};

// Applied field of a film (z component) for the device-side stage times.
struct FieldZ {
  int kind;
  double dz, amp, omega, rate;
};

// Kernel identifiers for the instrumentation.
enum KernelId {
  K_FILM_STENCIL = 0,
  K_FILM_ROWS_FWD_H,
  K_FILM_COLS,
  K_FILM_ROWS_INV_G,
  K_FILM_ROWS_FWD_G,
  K_FILM_ROWS_INV_UPD,
  K_BULK_CURL,
  K_BULK_EFIELD,
  K_BULK_HDOT_IN,
  K_BULK_X_FWD,
  K_BULK_Y_FWD,
  K_BULK_Z_PHI,
  K_BULK_Y_INV,
  K_BULK_X_INV_UPD,
  K_FINALIZE,
  K_MISC,
  K_RK,
  K_VJP,
  K_FILM_FINAL64,
  K_FILM_SPECTRAL,
  K_COUNT
};

struct ProfRec {
  hipEvent_t a, b;
  int kid;
  int iter;   // inner iteration index, -1 for per-call kernels
};

}  // namespace mag

struct mag_ctx {
  int dim = 0;
  int prec = 0;
  hipStream_t stream = nullptr;
  bool poisoned = false;
  std::string err;

  // grid
  bool grid_set = false, domain_set = false;
  int n[3] = {1, 1, 1};          // nx, ny, nz
  double L[3] = {1, 1, 1}, d[3] = {1, 1, 1};
  long long nnode = 0;            // nx*ny*nz
  int kx = 0;                     // nx/2 + 1
  long long nspec = 0;            // kx*ny*nz complex per component
  int ncomp = 1;                  // 1 (film) or 3 (bulk)

  // domain
  std::vector<uint8_t> h_mat;     // host copy of the material
  uint8_t *d_mat = nullptr;
  uint8_t *d_flags = nullptr;     // 2D: bit0 inside node; 3D: bits 0-2 inside faces, 3-5 inside edges
  long long nout = 0;             // number of free-space unknowns (nodes / edges)
  int box0[3] = {0, 0, 0}, box1[3] = {0, 0, 0};   // node box holding every inside face/edge/node

  // parameters
  double jc0 = 1, nexp = 19, e0 = 1, rho_out = 1;
  bool has_jc_map = false;
  void *d_jc = nullptr;           // per-cell jc (precision type)
  double *d_jc64 = nullptr;       // per-cell jc, double (VJP)
  double lambda = 0.7, tol = 2e-4;
  int max_inner = 100, fixed_iters = 0;

  // field
  int fkind = 0;
  double fdir[3] = {0, 0, 1}, famp = 1, fomega = 1, frate = 1;

  // workspace
  void *d_H = nullptr;            // iterate: film dh_z/dt on nodes; bulk dh/dt on edges (precision type)
  void *d_G = nullptr;            // film: G of (11) (precision type)
  void *d_S = nullptr;            // half spectrum, ncomp planes of kx*ny*nz complex
  void *d_w = nullptr;            // film: K1 and K2 applied to the free-space indicator (precision type)
  void *d_box = nullptr;          // bulk stencil scratch: j then e on the pruning box (precision type)
  long long boxvol = 0;
  int boxn[3] = {0, 0, 0};
  double *d_part = nullptr;       // per-block partial sums
  int npart = 0;
  mag::IterState *d_it = nullptr;
  mag::IterState *h_it = nullptr; // pinned
  void *d_tw = nullptr;           // twiddle tables (precision type)
  void *d_tw64 = nullptr;         // MAG_MIXED_FINAL64: the same tables in double
  mag::IterState *d_it64 = nullptr;   // MAG_MIXED_FINAL64: gate of the final evaluation
  double *d_w64 = nullptr;        // MAG_MIXED_FINAL64: w1 = K1 1_out in double
  int deriv = 0;                  // film derivatives: 0 staggered differences, 1 filtered spectral
  double dsigma = -1;             // spectral form: Gaussian width sigma (< 0: sqrt(dx^2 + dy^2))
  void *d_S2 = nullptr;           // spectral form: second half spectrum (j_y, then e_y), precision type
  void *d_jcn = nullptr;          // spectral form: per-node jc, NaN off superconducting nodes (precision type)
  unsigned long long jcn_gen = 0; // set-up generation d_jcn was computed for (0: none; gen starts at 1)
  void *d_S34 = nullptr;          // spectral VJP: two more half spectra (j_x, j_y), precision type
  double *d_cn = nullptr;         // spectral VJP: cotangent of the node jc
  mag::IterState *d_itv = nullptr;   // spectral VJP: state of its passes (C of the transposed iteration)
  double *d_filt = nullptr;       // spectral form: Gaussian factor per axis (kx entries, then ny)
  long long tw_off[4] = {0, 0, 0, 0};   // offsets: x half-length, y, z, x full-length (R2C post)
  double *d_sym = nullptr;        // per-axis symbol tables (double)
  long long sym_off[8] = {0};
  bool warm_valid = false;
  int last_iters = 1;

  // time stepping
  double *d_rk = nullptr;         // k1..k4, ytmp, ynew
  int rk_k1 = 0, rk_k4 = 3;       // which buffers currently hold k1 and k4
  bool fsal_valid = false;
  const double *fsal_state = nullptr;
  double fsal_t = 0;
  double *d_red = nullptr;        // reduction scratch for step control
  int nred = 0;


  // instrumentation
  bool debug_sync = false;        // MAG_DEBUG_SYNC=1: synchronise and check after every launch
  bool warm_enabled = true;   // start each RHS from the previous free-space solution
  bool rhs_async = false;      // the current mag_rhs returns without waiting (fixed count, no n_inner)
  bool async_pending = false;  // an asynchronous mag_rhs has not been checked yet
  bool prof_on = false;
  int prof_only = -1;   // record only this kernel id (-1: all)
  std::vector<mag::ProfRec> prof;
  std::vector<hipEvent_t> ev_pool;
  int cur_iter = -1;
  long long stat_rhs = 0, stat_inner = 0;   // mag_stats counts

  // device-driven integration (mag_integrate_captured)
  mag::StepCtl *d_sc = nullptr;
  mag::StepCtl *h_sc = nullptr;   // pinned, coherent
  hipStream_t cap_stream = nullptr;
  hipEvent_t cap_ev[2] = {nullptr, nullptr};
  hipGraphExec_t cap_exec = nullptr;
  const double *cap_state = nullptr;  // key of the instantiated graph
  int cap_chunk = 0;
  unsigned long long cap_gen = 0;
  unsigned long long gen = 1;         // bumped by every set_* call
  double prof_ms[mag::K_COUNT] = {0};
  int prof_cnt[mag::K_COUNT] = {0};
};

namespace mag {

int set_error(mag_ctx *c, int code, const char *fmt, ...);
int hip_check(mag_ctx *c, hipError_t e, const char *what);

#define MAG_HIP(ctx, expr)                                  \
  do {                                                      \
    hipError_t e_ = (expr);                                 \
    if (e_ != hipSuccess) return ::mag::hip_check(ctx, e_, #expr); \
  } while (0)

// instrumentation helpers
void prof_begin(mag_ctx *c, int kid, ProfRec *r);
void prof_end(mag_ctx *c, ProfRec *r);
void prof_drop_after(mag_ctx *c, int iters_done);

// Scoped launch timing: records events around the kernel when profiling is on.
struct ProfScope {
  mag_ctx *c;
  ProfRec r;
  ProfScope(mag_ctx *c_, int kid) : c(c_) { prof_begin(c, kid, &r); }
  ~ProfScope() { prof_end(c, &r); }
};

// Timing of a single kernel launch by the dispatch itself: the launch goes
// through hipExtLaunchKernelGGL with this record's events (null when the
// kernel is not being profiled), so the elapsed time is the kernel's own
// execution, without the marker packets that separate event records add.
void prof_launch_begin(mag_ctx *c, int kid, ProfRec *r);
void prof_launch_end(mag_ctx *c, ProfRec *r);
struct ProfLaunch {
  mag_ctx *c;
  ProfRec r;
  ProfLaunch(mag_ctx *c_, int kid) : c(c_) { prof_launch_begin(c, kid, &r); }
  ~ProfLaunch() { prof_launch_end(c, &r); }
  hipEvent_t start() const { return r.a; }
  hipEvent_t stop() const { return r.b; }
};
#define MAG_TIMED_LAUNCH(pl, K, G, B, S, STREAM, ...)                                   \
  do {                                                                                  \
    if ((pl).start())                                                                   \
      hipExtLaunchKernelGGL(K, G, B, S, STREAM, (pl).start(), (pl).stop(), 0, __VA_ARGS__); \
    else                                                                                \
      hipLaunchKernelGGL(K, G, B, S, STREAM, __VA_ARGS__);                               \
  } while (0)

// dimension-specific drivers
int film_alloc(mag_ctx *c);
int film_spectral_alloc(mag_ctx *c);   // the spectral form's buffers (forward and VJP), if not there yet
int film_domain(mag_ctx *c);
int film_rhs(mag_ctx *c, const double *state, double t, double *out, int *n_inner);
int film_observe(mag_ctx *c, const double *state, double t, double *hz, double *j, double *m);
int film_rhs_enqueue(mag_ctx *c, const double *state, double *out);
int film_rhs_vjp(mag_ctx *c, const double *state, double t, const double *out_bar,
                 double *state_bar, double *jc_bar);
int film_hz_transpose(mag_ctx *c, const double *hz_bar, double *state_bar);
int bulk_alloc(mag_ctx *c);
int bulk_domain(mag_ctx *c);
int bulk_rhs(mag_ctx *c, const double *state, double t, double *out, int *n_inner);
int bulk_observe(mag_ctx *c, const double *state, double t, double *hz, double *j, double *m);
int bulk_rhs_vjp(mag_ctx *c, const double *state, double t, const double *out_bar,
                 double *state_bar, double *jc_bar);

// applied field
void field_h(const mag_ctx *c, double t, double h[3]);
void field_hdot(const mag_ctx *c, double t, double hd[3]);

// shared launches (capi.hip, bulk.hip)
int run_finalize_stop(mag_ctx *c, int nparts);
int run_iter_init(mag_ctx *c, const IterState &is);
// which: 0 -> C = sum * inv_nout, 1 -> A = sum * inv_nout, 2 -> thr = sum * sum0;
// the partial sums start at d_part + first.
int run_finalize_mean(mag_ctx *c, int nparts, int which, int first = 0);
int run_to_double(mag_ctx *c, const void *src, double *dst, long long n);
int noalloc_setup();   // noalloc.hip: the current device's scratch address

}  // namespace mag
