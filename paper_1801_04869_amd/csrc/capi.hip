// C ABI of the library (declared in include/magfft.h): context life cycle,
// argument checks, twiddle tables, iteration finalizers, instrumentation and
// the Bogacki-Shampine 3(2) driver (the explicit pair behind Matlab's ode23,
// which the paper uses for the method of lines, Sec. 2.2).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <new>

#include "ctx.h"
#include "kern_common.h"

// The 3D (bulk) path is compiled for gfx950 but held off the GPU: its first
// GPU run ended in a memory fault whose cause has not been found (the CPU
// emulation of the same sources stays in bounds and matches the FP64 oracle).
// mag_set_grid refuses a 3D grid unless the build defines MAG_BULK_ENABLE,
// which only the CPU emulation build does.
#ifndef MAG_BULK_ENABLE
#define MAG_BULK_ENABLE 0
#endif

namespace mag {

int set_error(mag_ctx *c, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

int hip_check(mag_ctx *c, hipError_t e, const char *what) {
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    return set_error(c, MAG_E_NOMEM, "out of device memory in %s", what);
  }
  if (c) c->poisoned = true;
  return set_error(c, MAG_E_HIP, "HIP error '%s' in %s", hipGetErrorString(e), what);
}

void field_h(const mag_ctx *c, double t, double h[3]) {
  switch (c->fkind) {
    case MAG_FIELD_RAMP:
      for (int a = 0; a < 3; ++a) h[a] = c->fdir[a] * (c->frate * t);
      break;
    case MAG_FIELD_SINE:
      for (int a = 0; a < 3; ++a) h[a] = c->fdir[a] * (c->famp * std::sin(c->fomega * t));
      break;
    default:
      h[0] = c->famp * std::cos(c->fomega * t);
      h[1] = c->famp * std::sin(c->fomega * t);
      h[2] = 0.0;
  }
}

void field_hdot(const mag_ctx *c, double t, double hd[3]) {
  switch (c->fkind) {
    case MAG_FIELD_RAMP:
      for (int a = 0; a < 3; ++a) hd[a] = c->fdir[a] * c->frate;
      break;
    case MAG_FIELD_SINE:
      for (int a = 0; a < 3; ++a) hd[a] = c->fdir[a] * (c->famp * c->fomega * std::cos(c->fomega * t));
      break;
    default: {
      const double w = c->fomega;
      hd[0] = c->famp * w * -std::sin(w * t);
      hd[1] = c->famp * w * std::cos(w * t);
      hd[2] = 0.0;
    }
  }
}

// ---------------------------------------------------------------- instrumentation
static hipEvent_t pool_get(mag_ctx *c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

static const char *kNames[K_COUNT] = {
    "film_stencil", "film_rows_fwd_h", "film_cols", "film_rows_inv_g", "film_rows_fwd_g", "film_rows_inv_upd",
    "bulk_curl_box", "bulk_efield_box", "bulk_hdot_in", "bulk_x_fwd", "bulk_y_fwd", "bulk_z_phi",
    "bulk_y_inv", "bulk_x_inv", "finalize", "misc", "rk", "vjp", "film_final64",
    "film_spectral"};

void prof_begin(mag_ctx *c, int kid, ProfRec *r) {
  r->a = r->b = nullptr;
  r->kid = kid;
  r->iter = c->cur_iter;
  if (c->debug_sync) {
    fprintf(stderr, "[magfft] launch %s (iteration %d)\n", kNames[kid], c->cur_iter);
    fflush(stderr);
  }
  if (!c->prof_on || (c->prof_only >= 0 && kid != c->prof_only)) return;
  r->a = pool_get(c);
  r->b = pool_get(c);
  if (r->a) (void)hipEventRecord(r->a, c->stream);
}

void prof_end(mag_ctx *c, ProfRec *r) {
  if (c->debug_sync) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipGetLastError();
    fprintf(stderr, "[magfft]   %s -> %s\n", kNames[r->kid], e == hipSuccess ? "ok" : hipGetErrorString(e));
    fflush(stderr);
  }
  if (!c->prof_on || !r->a || !r->b) return;
  (void)hipEventRecord(r->b, c->stream);
  c->prof.push_back(*r);
}

void prof_launch_begin(mag_ctx *c, int kid, ProfRec *r) {
  r->a = r->b = nullptr;
  r->kid = kid;
  r->iter = c->cur_iter;
  if (c->debug_sync) {
    fprintf(stderr, "[magfft] launch %s (iteration %d)\n", kNames[kid], c->cur_iter);
    fflush(stderr);
  }
  if (!c->prof_on || (c->prof_only >= 0 && kid != c->prof_only)) return;
  r->a = pool_get(c);
  r->b = r->a ? pool_get(c) : nullptr;
  if (!r->b) r->a = nullptr;
}

void prof_launch_end(mag_ctx *c, ProfRec *r) {
  if (c->debug_sync) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipGetLastError();
    fprintf(stderr, "[magfft]   %s -> %s\n", kNames[r->kid], e == hipSuccess ? "ok" : hipGetErrorString(e));
    fflush(stderr);
  }
  if (!c->prof_on || !r->a || !r->b) return;
  c->prof.push_back(*r);
}

// Called after an RHS: launches of iterations >= iters_done found `done` set
// and returned at once; drop them (they are the newest records).
void prof_drop_after(mag_ctx *c, int iters_done) {
  if (!c->prof_on) return;
  while (!c->prof.empty() && c->prof.back().iter >= iters_done) {
    c->ev_pool.push_back(c->prof.back().a);
    c->ev_pool.push_back(c->prof.back().b);
    c->prof.pop_back();
  }
}

static void prof_clear(mag_ctx *c) {
  for (auto &r : c->prof) {
    c->ev_pool.push_back(r.a);
    c->ev_pool.push_back(r.b);
  }
  c->prof.clear();
  for (int k = 0; k < K_COUNT; ++k) {
    c->prof_ms[k] = 0;
    c->prof_cnt[k] = 0;
  }
}

// ---------------------------------------------------------------- finalizers
namespace {

__device__ __forceinline__ double fixed_order_sum(const double *__restrict__ part, int n, double *sh) {
  double s = 0.0;
  int i = threadIdx.x;
  // eight loads in flight per thread, added in index order
  for (; i + 7 * 256 < n; i += 8 * 256) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[i + u * 256];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; i < n; i += 256) s += part[i];
  return block_sum<256>(s, sh);
}

// Stop test of the inner iteration.  The updated state is also written to
// the context's pinned host mirror, which the host reads after synchronising
// the stream (no separate device-to-host copy).
__global__ void __launch_bounds__(256) finalize_stop_k(const double *__restrict__ part, int n, IterState *it,
                                                       IterState *mirror) {
  if (it->done) return;
  __shared__ double sh[256];
  const double s = fixed_order_sum(part, n, sh);
  if (threadIdx.x == 0) {
    IterState v = *it;
    const double r = s * v.inv_nout;
    v.r = r;
    v.iters += 1;
    if (!isfinite(r)) {
      v.done = 2;
      v.fail = 1;
    } else if (v.fixed > 0) v.done = v.iters >= v.fixed ? 1 : 0;
    else v.done = r < v.thr ? 1 : 0;
    *it = v;
    *mirror = v;
  }
}

// Reset of the iteration state at the start of a right-hand side; keep_fail
// carries the failure flag of the evaluations queued before it.
__global__ void __launch_bounds__(64) iter_init_k(IterState *it, IterState *mirror, IterState v, int keep_fail) {
  if (threadIdx.x == 0) {
    if (keep_fail) v.fail = it->fail;
    *it = v;
    *mirror = v;
  }
}

__global__ void __launch_bounds__(256) finalize_mean_k(const double *__restrict__ part, int n, IterState *it,
                                                       int which) {
  if (it->done) return;
  __shared__ double sh[256];
  const double s = fixed_order_sum(part, n, sh);
  if (threadIdx.x == 0) {
    if (which == 0) it->C = s * it->inv_nout;
    else if (which == 1) it->A = s * it->inv_nout;
    else it->thr = s * it->sum0;   // stop threshold from a sum (sum0 holds the factor)
  }
}

// out = y + h * sum_i w_i k_i  (nk <= 3)
__global__ void __launch_bounds__(256) rk_axpy_k(double *__restrict__ out, const double *__restrict__ y,
                                                 const double *__restrict__ k0, const double *__restrict__ k1,
                                                 const double *__restrict__ k2, double w0, double w1, double w2,
                                                 int nk, double h, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = w0 * k0[i];
  if (nk > 1) s += w1 * k1[i];
  if (nk > 2) s += w2 * k2[i];
  out[i] = y[i] + h * s;
}

// out = a x + b y (y may be NULL); out may alias x or y.
__global__ void __launch_bounds__(256) lincomb_k(double *out, double a, const double *x, double b, const double *y,
                                                 long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double v = a * x[i] + (y ? b * y[i] : 0.0);
  out[i] = v;
}

// per-block max of |h sum e_i k_i| / max(rtol max(|y|,|ynew|), atol); non-finite -> inf
__global__ void __launch_bounds__(256) rk_errnorm_k(const double *__restrict__ k1, const double *__restrict__ k2,
                                                    const double *__restrict__ k3, const double *__restrict__ k4,
                                                    double e1, double e2, double e3, double e4, double h,
                                                    const double *__restrict__ y, const double *__restrict__ yn,
                                                    double rtol, double atol, long long n,
                                                    double *__restrict__ part) {
  __shared__ double sh[256];
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    const double err = h * (e1 * k1[i] + e2 * k2[i] + e3 * k3[i] + e4 * k4[i]);
    const double sc = fmax(rtol * fmax(fabs(y[i]), fabs(yn[i])), atol);
    v = fabs(err) / sc;
    if (!isfinite(v)) v = INFINITY;
  }
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// per-block max of |f| / max(|y|, thr)
__global__ void __launch_bounds__(256) rk_ratio_k(const double *__restrict__ f, const double *__restrict__ y,
                                                  double thr, long long n, double *__restrict__ part) {
  __shared__ double sh[256];
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    v = fabs(f[i]) / fmax(fabs(y[i]), thr);
    if (!isfinite(v)) v = INFINITY;
  }
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// ---------------------------------------------------------------- device-side step control
// Kernels of a step attempt whose t and h live in device memory (StepCtl):
// the same arithmetic as the host-driven step (stage times t + c h, stage
// states y + (a h) k, error norm, controller), so that a run of attempts can
// be captured in one graph and replayed without host decisions.  Every kernel
// returns at once when the run is finished.

__device__ __forceinline__ double field_hdot_z(const FieldZ &f, double t) {
  if (f.kind == MAG_FIELD_RAMP) return f.dz * f.rate;
  if (f.kind == MAG_FIELD_SINE) return f.dz * (f.amp * f.omega * cos(f.omega * t));
  return 0.0;   // the rotating field lies in the film plane
}

// Iteration state of the stage at t + cs h: dh_e/dt there, the stop threshold
// tol max(|dh_e/dt|, 1), the failure flag kept from the earlier stages of the
// attempt (keep_fail), done when the run is finished.
__global__ void __launch_bounds__(64) stage_init_k(IterState *it, IterState *mirror, const StepCtl *sc, FieldZ f,
                                                   double cs, IterState base, double tol, int keep_fail) {
  if (threadIdx.x != 0) return;
  IterState v = base;
  // the first stage of an attempt after a failed one restarts cold (as the
  // host-driven step drops its warm start after a failure)
  if (keep_fail) v.fail = it->fail;
  else v.cold = it->fail;
  const double ts = sc->t + cs * sc->h;
  const double hde = field_hdot_z(f, ts);
  v.hde = hde;
  v.thr = tol * (fabs(hde) > 1.0 ? fabs(hde) : 1.0);
  if (sc->finished) v.done = 1;
  *it = v;
  *mirror = v;
}

// out = y + (hfac h) sum_i w_i k_i  (nk <= 3), h from the step record.
__global__ void __launch_bounds__(256) rk_axpy_sc_k(double *__restrict__ out, const double *__restrict__ y,
                                                    const double *__restrict__ k0, const double *__restrict__ k1,
                                                    const double *__restrict__ k2, double w0, double w1, double w2,
                                                    int nk, double hfac, const StepCtl *__restrict__ sc,
                                                    long long n) {
  if (sc->finished) return;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double h = hfac * sc->h;
  double s = w0 * k0[i];
  if (nk > 1) s += w1 * k1[i];
  if (nk > 2) s += w2 * k2[i];
  out[i] = y[i] + h * s;
}

// Per-block max of the scaled error (as rk_errnorm_k), h, rtol and atol from
// the step record.  kErrNpt entries per work-item, 256 apart, so that the
// accept kernel has few block maxima to combine.
constexpr int kErrNpt = 8;
__global__ void __launch_bounds__(256) rk_errnorm_sc_k(const double *__restrict__ k1, const double *__restrict__ k2,
                                                       const double *__restrict__ k3, const double *__restrict__ k4,
                                                       double e1, double e2, double e3, double e4,
                                                       const double *__restrict__ y, const double *__restrict__ yn,
                                                       const StepCtl *__restrict__ sc, long long n,
                                                       double *__restrict__ part) {
  __shared__ double sh[256];
  if (sc->finished) return;
  const double h = sc->h, rtol = sc->rtol, atol = sc->atol;
  const long long i0 = (long long)blockIdx.x * (256 * kErrNpt) + threadIdx.x;
  double v = 0.0;
#pragma unroll
  for (int u = 0; u < kErrNpt; ++u) {
    const long long i = i0 + (long long)u * 256;
    if (i < n) {
      const double err = h * (e1 * k1[i] + e2 * k2[i] + e3 * k3[i] + e4 * k4[i]);
      const double sc_ = fmax(rtol * fmax(fabs(y[i]), fabs(yn[i])), atol);
      double w = fabs(err) / sc_;
      if (!isfinite(w)) w = INFINITY;
      v = fmax(v, w);
    }
  }
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Accept or reject the attempt: error norm = max of the block maxima; a
// failed stage (non-finite residual, sticky flag) rejects with h / 2 (Sec.
// 2.2 reduces the step when gdot blows up); otherwise the controller of the
// host-driven step.  Then the end-time clip and the underflow check that the
// host loop applies before an attempt.
__global__ void __launch_bounds__(256) step_accept_k(StepCtl *sc, StepCtl *mirror, const double *__restrict__ part,
                                                     int nb, const IterState *__restrict__ it) {
  __shared__ double sh[256];
  if (sc->finished) {
    if (threadIdx.x == 0) {
      sc->commit = 0;
      *mirror = *sc;
    }
    return;
  }
  // eight block maxima in flight per work-item
  double m = 0.0;
  for (int i0 = threadIdx.x; i0 < nb; i0 += 256 * 8) {
    double w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) w[u] = i0 + u * 256 < nb ? part[i0 + u * 256] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) m = fmax(m, w[u]);
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  StepCtl v = *sc;
  const double en = sh[0];
  const double h = v.h;
  v.err = en;
  if (it->fail == 0 && en <= 1.0) {
    v.t = v.t + h;
    const double fac = en == 0.0 ? 5.0 : fmin(5.0, fmax(0.2, 0.8 * pow(en, -1.0 / 3.0)));
    v.h = h * fac;
    v.accepted += 1;
    v.commit = 1;
  } else {
    const double fac = it->fail ? 0.5 : fmax(0.2, 0.8 * pow(en, -1.0 / 3.0));
    v.h = h * fac;
    v.rejected += 1;
    v.commit = 0;
  }
  if (!(v.t < v.t_end)) {
    v.finished = 1;
  } else {
    if (1.1 * v.h >= v.t_end - v.t) v.h = v.t_end - v.t;
    if (v.h <= 16.0 * 2.220446049250313e-16 * fmax(fabs(v.t), 1.0)) {
      v.status = MAG_STEP_UNDERFLOW;
      v.finished = 1;
    }
  }
  *sc = v;
  *mirror = v;
}

// An accepted attempt: y <- y_new and k1 <- k4 (first same as last).
__global__ void __launch_bounds__(256) step_commit_k(double *__restrict__ y, const double *__restrict__ yn,
                                                     double *__restrict__ k1, const double *__restrict__ k4,
                                                     const StepCtl *__restrict__ sc, long long n) {
  if (!sc->commit) return;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  y[i] = yn[i];
  k1[i] = k4[i];
}

template <typename T>
__global__ void fill_twiddles(cx<T> *dst, const double *src, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = {(T)src[2 * i], (T)src[2 * i + 1]};
}

template <typename T>
__global__ void scale_jc(const double *__restrict__ src, T *__restrict__ dst, double *__restrict__ d64,
                         double jc0, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    const double v = jc0 * src[i];
    dst[i] = (T)v;
    d64[i] = v;
  }
}

}  // namespace

int run_finalize_stop(mag_ctx *c, int nparts) {
  ProfScope ps(c, K_FINALIZE);
  hipLaunchKernelGGL(finalize_stop_k, dim3(1), dim3(256), 0, c->stream, c->d_part, nparts, c->d_it, c->h_it);
  return MAG_OK;
}

int run_iter_init(mag_ctx *c, const IterState &is) {
  ProfScope ps(c, K_FINALIZE);
  // an evaluation queued behind an unchecked asynchronous one keeps its failure flag
  hipLaunchKernelGGL(iter_init_k, dim3(1), dim3(64), 0, c->stream, c->d_it, c->h_it, is, c->async_pending ? 1 : 0);
  MAG_HIP(c, hipGetLastError());
  return MAG_OK;
}

int run_finalize_mean(mag_ctx *c, int nparts, int which, int first) {
  ProfScope ps(c, K_FINALIZE);
  hipLaunchKernelGGL(finalize_mean_k, dim3(1), dim3(256), 0, c->stream, c->d_part + first, nparts, c->d_it, which);
  return MAG_OK;
}

static int ensure_red(mag_ctx *c, long long n) {
  const int nb = (int)((n + 255) / 256);
  if (c->nred < nb) {
    if (c->d_red) (void)hipFree(c->d_red);
    c->d_red = nullptr;
    MAG_HIP(c, hipMalloc(&c->d_red, (size_t)nb * sizeof(double)));
    c->nred = nb;
  }
  return MAG_OK;
}

static int host_max(mag_ctx *c, int nb, double *out) {
  std::vector<double> v(nb);
  MAG_HIP(c, hipMemcpyAsync(v.data(), c->d_red, nb * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  MAG_HIP(c, hipStreamSynchronize(c->stream));
  double m = 0.0;
  for (double x : v) m = std::max(m, x);
  *out = m;
  return MAG_OK;
}

}  // namespace mag

using namespace mag;

// ==================================================================== C ABI
extern "C" {

static bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }
// three times a power of two in [lo, hi]
static bool pow2x3_in(int n, int lo, int hi) { return n % 3 == 0 && pow2_in(n / 3, (lo + 2) / 3, hi / 3); }

static void free_all(mag_ctx *c) {
  void *ptrs[] = {c->d_mat, c->d_flags, c->d_jc, c->d_jc64, c->d_H, c->d_G, c->d_S, c->d_box,
                  c->d_part, c->d_it, c->d_tw, c->d_sym, c->d_rk, c->d_red, c->d_w,
                  c->d_tw64, c->d_it64, c->d_w64, c->d_S2, c->d_jcn, c->d_S34, c->d_cn, c->d_itv,
                  c->d_filt};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  c->d_mat = c->d_flags = nullptr;
  c->d_jc = c->d_H = c->d_G = c->d_S = c->d_box = c->d_tw = c->d_w = c->d_tw64 = nullptr;
  c->d_it64 = nullptr;
  c->d_w64 = nullptr;
  c->d_S2 = c->d_jcn = c->d_S34 = nullptr;
  c->d_cn = c->d_filt = nullptr;
  c->d_itv = nullptr;
  c->d_jc64 = c->d_part = c->d_sym = c->d_rk = c->d_red = nullptr;
  c->d_it = nullptr;
  c->nred = 0;
}

int mag_create(mag_ctx **out, int dim, int precision, void *hip_stream) {
  if (!out) return MAG_E_ARG;
  *out = nullptr;
  if (dim != 2 && dim != 3) return MAG_E_ARG;
  if (precision != MAG_FP64 && precision != MAG_MIXED && precision != MAG_MIXED_FINAL64) return MAG_E_ARG;
  if (precision == MAG_MIXED_FINAL64 && dim != 2) return MAG_E_ARG;
  mag_ctx *c = new (std::nothrow) mag_ctx();
  if (!c) return MAG_E_NOMEM;
  c->dim = dim;
  c->prec = precision;
  c->ncomp = dim == 3 ? 3 : 1;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (dim == 3) c->tol = 1e-4;
  const char *dbg = getenv("MAG_DEBUG_SYNC");
  c->debug_sync = dbg && dbg[0] == '1';
  // coherent pinned memory: kernels write the iteration state straight into it
  if (hipHostMalloc(&c->h_it, sizeof(IterState), hipHostMallocCoherent) != hipSuccess) {
    delete c;
    return MAG_E_HIP;
  }
  if (hipMalloc(&c->d_it, sizeof(IterState)) != hipSuccess) {
    (void)hipHostFree(c->h_it);
    delete c;
    return MAG_E_NOMEM;
  }
  // set-up of the allocation-free entry point on this device (retried by
  // its first call if it fails here)
  (void)noalloc_setup();
  *out = c;
  return MAG_OK;
}

static void release_capture(mag_ctx *c) {
  if (c->cap_stream) (void)hipStreamSynchronize(c->cap_stream);
  if (c->cap_exec) (void)hipGraphExecDestroy(c->cap_exec);
  c->cap_exec = nullptr;
  c->cap_state = nullptr;
}

void mag_destroy(mag_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  release_capture(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (hipEvent_t e : c->cap_ev)
    if (e) (void)hipEventDestroy(e);
  if (c->d_sc) (void)hipFree(c->d_sc);
  if (c->h_sc) (void)hipHostFree(c->h_sc);
  prof_clear(c);
  for (hipEvent_t e : c->ev_pool)
    if (e) (void)hipEventDestroy(e);
  free_all(c);
  if (c->h_it) (void)hipHostFree(c->h_it);
  delete c;
}

const char *mag_last_error(const mag_ctx *c) { return c ? c->err.c_str() : "null context"; }

#define CHECK_CTX(c)                                                     \
  do {                                                                   \
    if (!(c)) return MAG_E_ARG;                                          \
    if ((c)->poisoned) return set_error(c, MAG_E_HIP, "context unusable after a HIP error"); \
  } while (0)

int mag_set_grid(mag_ctx *c, int nx, int ny, int nz, double Lx, double Ly, double Lz) {
  CHECK_CTX(c);
  ++c->gen;   // a captured step graph bakes the set-up in
  if (c->dim == 3 && (!pow2_in(nx, 16, 2048) || !pow2_in(ny, 16, 2048)))
    return set_error(c, MAG_E_ARG, "nx, ny must be powers of two in [16, 2048]");
  if (c->dim == 2 && (!(pow2_in(nx, 16, 2048) || pow2x3_in(nx, 48, 768)) ||
                      !(pow2_in(ny, 16, 2048) || pow2x3_in(ny, 48, 768))))
    return set_error(c, MAG_E_ARG,
                     "film grid: nx, ny powers of two in [16, 2048] or three times one in [48, 768]");
  if (c->dim == 2 && nz != 1) return set_error(c, MAG_E_ARG, "nz must be 1 for a film");
  if (c->dim == 3 && !pow2_in(nz, 16, 2048)) return set_error(c, MAG_E_ARG, "nz must be a power of two in [16, 2048]");
  if (!(Lx > 0) || !(Ly > 0) || (c->dim == 3 && !(Lz > 0))) return set_error(c, MAG_E_ARG, "box half-lengths must be positive");
  if (c->dim == 3 && !MAG_BULK_ENABLE)
    return set_error(c, MAG_E_STATE,
                     "the 3D path is disabled (held off the GPU after an unexplained memory fault; "
                     "MAG_BULK_ENABLE compiles it in)");
  MAG_HIP(c, hipStreamSynchronize(c->stream));
  release_capture(c);
  IterState *keep_it = c->d_it;
  c->d_it = nullptr;
  free_all(c);
  c->d_it = keep_it;
  c->grid_set = c->domain_set = false;
  c->has_jc_map = false;
  c->n[0] = nx;
  c->n[1] = ny;
  c->n[2] = nz;
  c->L[0] = Lx;
  c->L[1] = Ly;
  c->L[2] = c->dim == 3 ? Lz : 1.0;
  for (int a = 0; a < 3; ++a) c->d[a] = 2.0 * c->L[a] / c->n[a];
  c->nnode = (long long)nx * ny * nz;
  c->kx = nx / 2 + 1;
  c->nspec = (long long)c->kx * ny * nz;
  c->warm_valid = false;
  c->fsal_valid = false;
  c->last_iters = 1;
  int rc = c->dim == 3 ? bulk_alloc(c) : film_alloc(c);
  if (rc) return rc;
  // twiddles exp(-2 pi i m / n): x half length, y, z, x full length
  std::vector<double> tw;
  auto add = [&](int n, int slot) {
    c->tw_off[slot] = (long long)tw.size() / 2;
    for (int m = 0; m < n; ++m) {
      const double a = -2.0 * M_PI * (double)m / (double)n;
      tw.push_back(std::cos(a));
      tw.push_back(std::sin(a));
    }
  };
  add(nx / 2, 0);
  add(ny, 1);
  add(c->dim == 3 ? nz : 1, 2);
  add(nx, 3);
  const long long ntw = (long long)tw.size() / 2;
  const size_t ts = c->prec == MAG_FP64 ? 8 : 4;
  double *tmp = nullptr;
  MAG_HIP(c, hipMalloc(&c->d_tw, ntw * 2 * ts));
  MAG_HIP(c, hipMalloc(&tmp, tw.size() * sizeof(double)));
  MAG_HIP(c, hipMemcpy(tmp, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice));
  if (c->prec == MAG_MIXED_FINAL64) MAG_HIP(c, hipMalloc(&c->d_tw64, ntw * 2 * sizeof(double)));
  {
  ProfScope ps(c, K_MISC);
  if (c->prec == MAG_FP64)
    hipLaunchKernelGGL((fill_twiddles<double>), dim3((unsigned)((ntw + 255) / 256)), dim3(256), 0, c->stream,
                       reinterpret_cast<cx<double> *>(c->d_tw), tmp, ntw);
  else
    hipLaunchKernelGGL((fill_twiddles<float>), dim3((unsigned)((ntw + 255) / 256)), dim3(256), 0, c->stream,
                       reinterpret_cast<cx<float> *>(c->d_tw), tmp, ntw);
  if (c->d_tw64)
    hipLaunchKernelGGL((fill_twiddles<double>), dim3((unsigned)((ntw + 255) / 256)), dim3(256), 0, c->stream,
                       reinterpret_cast<cx<double> *>(c->d_tw64), tmp, ntw);
  }
  MAG_HIP(c, hipGetLastError());
  MAG_HIP(c, hipStreamSynchronize(c->stream));
  MAG_HIP(c, hipFree(tmp));
  // per-cell jc (uniform until set_params gives a map)
  MAG_HIP(c, hipMalloc(&c->d_jc, c->nnode * ts));
  MAG_HIP(c, hipMalloc(&c->d_jc64, c->nnode * sizeof(double)));
  c->grid_set = true;
  return MAG_OK;
}

int mag_set_domain(mag_ctx *c, const uint8_t *material) {
  CHECK_CTX(c);
  ++c->gen;   // a captured step graph bakes the set-up in
  if (!c->grid_set) return set_error(c, MAG_E_STATE, "mag_set_domain before mag_set_grid");
  if (!material) return set_error(c, MAG_E_ARG, "material is NULL");
  std::vector<uint8_t> m(c->nnode);
  MAG_HIP(c, hipStreamSynchronize(c->stream));
  MAG_HIP(c, hipMemcpy(m.data(), material, c->nnode, hipMemcpyDefault));
  for (uint8_t v : m)
    if (v > 2) return set_error(c, MAG_E_ARG, "material codes must be 0, 1 or 2");
  c->h_mat.swap(m);
  int rc = c->dim == 3 ? bulk_domain(c) : film_domain(c);
  if (rc) {
    c->domain_set = false;
    return rc;
  }
  c->domain_set = true;
  c->fsal_valid = false;
  return MAG_OK;
}

int mag_set_params(mag_ctx *c, const double *jc_map, double jc0, double n, double e0, double rho_out) {
  CHECK_CTX(c);
  ++c->gen;   // a captured step graph bakes the set-up in
  if (!c->grid_set) return set_error(c, MAG_E_STATE, "mag_set_params before mag_set_grid");
  if (!(n >= 1.0) || !(jc0 > 0) || !(e0 > 0) || !(rho_out >= 0) || !std::isfinite(n) || !std::isfinite(jc0))
    return set_error(c, MAG_E_ARG, "need n >= 1, jc0 > 0, e0 > 0, rho_out >= 0");
  if (jc_map) {
    std::vector<double> h(c->nnode);
    MAG_HIP(c, hipStreamSynchronize(c->stream));
    MAG_HIP(c, hipMemcpy(h.data(), jc_map, c->nnode * sizeof(double), hipMemcpyDefault));
    for (double v : h)
      if (!(v > 0) || !std::isfinite(v)) return set_error(c, MAG_E_ARG, "jc_map entries must be positive and finite");
    double *tmp = nullptr;
    MAG_HIP(c, hipMalloc(&tmp, c->nnode * sizeof(double)));
    MAG_HIP(c, hipMemcpy(tmp, h.data(), c->nnode * sizeof(double), hipMemcpyHostToDevice));
    const unsigned nb = (unsigned)((c->nnode + 255) / 256);
    ProfScope ps(c, K_MISC);
    if (c->prec == MAG_FP64)
      hipLaunchKernelGGL((scale_jc<double>), dim3(nb), dim3(256), 0, c->stream, tmp,
                         reinterpret_cast<double *>(c->d_jc), c->d_jc64, jc0, c->nnode);
    else
      hipLaunchKernelGGL((scale_jc<float>), dim3(nb), dim3(256), 0, c->stream, tmp,
                         reinterpret_cast<float *>(c->d_jc), c->d_jc64, jc0, c->nnode);
    MAG_HIP(c, hipGetLastError());
    MAG_HIP(c, hipStreamSynchronize(c->stream));
    MAG_HIP(c, hipFree(tmp));
  }
  c->has_jc_map = jc_map != nullptr;
  c->jc0 = jc0;
  c->nexp = n;
  c->e0 = e0;
  c->rho_out = rho_out;
  c->fsal_valid = false;
  return MAG_OK;
}

int mag_set_solver(mag_ctx *c, double lambda, double inner_tol, int max_inner, int fixed_iters) {
  CHECK_CTX(c);
  ++c->gen;   // a captured step graph bakes the set-up in
  if (!(lambda > 0) || !(inner_tol >= 0) || max_inner < 1 || fixed_iters < 0 || max_inner > 100000 ||
      fixed_iters > 100000)
    return set_error(c, MAG_E_ARG, "need lambda > 0, inner_tol >= 0, 1 <= max_inner, fixed_iters >= 0");
  c->lambda = lambda;
  c->tol = inner_tol;
  c->max_inner = max_inner;
  c->fixed_iters = fixed_iters;
  c->fsal_valid = false;
  return MAG_OK;
}

int mag_set_field(mag_ctx *c, int kind, const double dir[3], double amp, double omega, double rate) {
  CHECK_CTX(c);
  ++c->gen;   // a captured step graph bakes the set-up in
  if (kind < 0 || kind > 2) return set_error(c, MAG_E_ARG, "unknown field kind");
  if ((kind != MAG_FIELD_ROTATE) && !dir) return set_error(c, MAG_E_ARG, "dir is NULL");
  c->fkind = kind;
  if (dir)
    for (int a = 0; a < 3; ++a) c->fdir[a] = dir[a];
  c->famp = amp;
  c->fomega = omega;
  c->frate = rate;
  c->fsal_valid = false;
  return MAG_OK;
}

static int ready(mag_ctx *c) {
  if (!c->grid_set) return set_error(c, MAG_E_STATE, "grid not set");
  if (!c->domain_set) return set_error(c, MAG_E_STATE, "domain not set");
  return MAG_OK;
}

static int rhs_impl(mag_ctx *c, const double *state, double t, double *out, int *n_inner) {
  if (!c->warm_enabled) c->warm_valid = false;
  int it = 0;
  const int rc = c->dim == 3 ? bulk_rhs(c, state, t, out, &it) : film_rhs(c, state, t, out, &it);
  if (rc >= 0) {
    c->stat_rhs += 1;
    c->stat_inner += it;
  }
  if (n_inner) *n_inner = it;
  return rc;
}

static int rhs_vjp_impl(mag_ctx *c, const double *state, double t, const double *out_bar, double *state_bar,
                        double *jc_bar) {
  return c->dim == 3 ? bulk_rhs_vjp(c, state, t, out_bar, state_bar, jc_bar)
                     : film_rhs_vjp(c, state, t, out_bar, state_bar, jc_bar);
}

int mag_rhs(mag_ctx *c, const double *state, double t, double *out, int *n_inner) {
  CHECK_CTX(c);
  int rc = ready(c);
  if (rc) return rc;
  if (!state || !out) return set_error(c, MAG_E_ARG, "state/out is NULL");
  if (state == out) return set_error(c, MAG_E_ARG, "out must not alias state");
  if (!std::isfinite(t)) return set_error(c, MAG_E_ARG, "t is not finite");
  c->fsal_valid = false;
  c->rhs_async = n_inner == nullptr && c->fixed_iters > 0 && c->dim == 2;
  rc = rhs_impl(c, state, t, out, n_inner);
  c->rhs_async = false;
  return rc;
}

int mag_rhs_status(mag_ctx *c, int *n_inner) {
  CHECK_CTX(c);
  MAG_HIP(c, hipStreamSynchronize(c->stream));
  if (n_inner) *n_inner = c->h_it->iters;
  if (!c->async_pending) return MAG_OK;
  c->async_pending = false;
  if (c->h_it->fail || c->h_it->done == 2 || !std::isfinite(c->h_it->r) || !std::isfinite(c->h_it->C)) {
    c->warm_valid = false;
    return set_error(c, MAG_E_NUMERIC, "non-finite residual");
  }
  return MAG_OK;
}

int mag_reset_warm_start(mag_ctx *c) {
  CHECK_CTX(c);
  c->warm_valid = false;
  c->last_iters = 1;
  return MAG_OK;
}

int mag_set_derivatives(mag_ctx *c, int mode, double sigma) {
  CHECK_CTX(c);
  if (c->dim != 2) return set_error(c, MAG_E_ARG, "the spectral form is a film option");
  if (mode != MAG_DERIV_STAGGERED && mode != MAG_DERIV_SPECTRAL)
    return set_error(c, MAG_E_ARG, "mode must be MAG_DERIV_STAGGERED or MAG_DERIV_SPECTRAL");
  if (!std::isfinite(sigma)) return set_error(c, MAG_E_ARG, "sigma must be finite");
  ++c->gen;   // a captured step graph bakes the set-up in
  MAG_HIP(c, hipStreamSynchronize(c->stream));
  c->deriv = mode;
  c->dsigma = sigma;
  c->warm_valid = false;
  c->fsal_valid = false;
  // buffers and the filter tables of this sigma (the grid's set-up does the
  // same when it comes later)
  if (mode == MAG_DERIV_SPECTRAL && c->grid_set)
    if (int rc = film_spectral_alloc(c)) return rc;
  return MAG_OK;
}

int mag_set_warm_start(mag_ctx *c, int on) {
  CHECK_CTX(c);
  c->warm_enabled = on != 0;
  if (!c->warm_enabled) c->warm_valid = false;
  return MAG_OK;
}

// ---------------------------------------------------------------- time stepping
static const double kRkC2 = 0.5, kRkC3 = 0.75, kA21 = 0.5, kA32 = 0.75;
static const double kB1 = 2.0 / 9.0, kB2 = 1.0 / 3.0, kB3 = 4.0 / 9.0;
static const double kE1 = -5.0 / 72.0, kE2 = 1.0 / 12.0, kE3 = 1.0 / 9.0, kE4 = -1.0 / 8.0;

static long long state_len(const mag_ctx *c) { return c->nnode * c->ncomp; }

static int ensure_rk(mag_ctx *c) {
  if (c->d_rk) return MAG_OK;
  MAG_HIP(c, hipMalloc(&c->d_rk, 6 * state_len(c) * sizeof(double)));
  return MAG_OK;
}

static double *rk_buf(mag_ctx *c, int i) { return c->d_rk + (long long)i * state_len(c); }

// buffers: 0..3 = k1..k4 (k1/k4 roles swap after each accepted step), 4 = ytmp, 5 = ynew

static int launch_axpy(mag_ctx *c, double *out, const double *y, const double *k0, const double *k1,
                       const double *k2, double w0, double w1, double w2, int nk, double h) {
  const long long n = state_len(c);
  ProfScope ps(c, K_RK);
  hipLaunchKernelGGL(rk_axpy_k, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, out, y, k0,
                     k1 ? k1 : k0, k2 ? k2 : k0, w0, w1, w2, nk, h, n);
  MAG_HIP(c, hipGetLastError());
  return MAG_OK;
}

// Stage evaluations k2..k4 of a step with a fixed inner count (film) are
// enqueued without a host wait: nothing in them is data-dependent control.
// A stage whose residual turns non-finite stops writing its output, so the
// failure flag of the iteration state is sticky along the queued stages (the
// reset of each later stage keeps it) and the step's one synchronisation
// checks it.  With the stop test every evaluation keeps its host poll.
static int stage_rhs(mag_ctx *c, const double *y, double t, double *k) {
  c->rhs_async = c->fixed_iters > 0 && c->dim == 2;
  const int rc = rhs_impl(c, y, t, k, nullptr);
  c->rhs_async = false;
  return rc;
}

// After a synchronisation: the status of the stages enqueued by stage_rhs.
static int stages_status(mag_ctx *c) {
  if (!c->async_pending) return MAG_OK;
  c->async_pending = false;
  if (c->h_it->fail || c->h_it->done == 2 || !std::isfinite(c->h_it->r) || !std::isfinite(c->h_it->C)) {
    c->warm_valid = false;
    return set_error(c, MAG_E_NUMERIC, "non-finite residual");
  }
  return MAG_OK;
}

static int step_impl(mag_ctx *c, double *state, double *t, double *dt, double rtol, double atol, int *accepted) {
  int rc = ensure_rk(c);
  if (rc) return rc;
  const long long n = state_len(c);
  double *k1 = rk_buf(c, c->rk_k1), *k4 = rk_buf(c, c->rk_k4);
  double *k2 = rk_buf(c, 1), *k3 = rk_buf(c, 2), *yt = rk_buf(c, 4), *yn = rk_buf(c, 5);
  const double h = *dt;
  *accepted = 0;
  if (!(c->fsal_valid && c->fsal_state == state && c->fsal_t == *t)) {
    rc = rhs_impl(c, state, *t, k1, nullptr);
    if (rc != MAG_OK) return rc;
    c->fsal_valid = true;
    c->fsal_state = state;
    c->fsal_t = *t;
  }
  auto failed = [&](int st) { return st == MAG_NOT_CONVERGED || st == MAG_E_NUMERIC; };
  if ((rc = launch_axpy(c, yt, state, k1, nullptr, nullptr, 1.0, 0, 0, 1, kA21 * h))) return rc;
  rc = stage_rhs(c, yt, *t + kRkC2 * h, k2);
  if (failed(rc)) {
    *dt = 0.5 * h;
    return MAG_OK;
  }
  if (rc) return rc;
  if ((rc = launch_axpy(c, yt, state, k2, nullptr, nullptr, 1.0, 0, 0, 1, kA32 * h))) return rc;
  rc = stage_rhs(c, yt, *t + kRkC3 * h, k3);
  if (failed(rc)) {
    *dt = 0.5 * h;
    return MAG_OK;
  }
  if (rc) return rc;
  if ((rc = launch_axpy(c, yn, state, k1, k2, k3, kB1, kB2, kB3, 3, h))) return rc;
  rc = stage_rhs(c, yn, *t + h, k4);
  if (failed(rc)) {
    *dt = 0.5 * h;
    return MAG_OK;
  }
  if (rc) return rc;
  if ((rc = ensure_red(c, n))) return rc;
  const int nb = (int)((n + 255) / 256);
  {
    ProfScope ps(c, K_RK);
    hipLaunchKernelGGL(rk_errnorm_k, dim3(nb), dim3(256), 0, c->stream, k1, k2, k3, k4, kE1, kE2, kE3, kE4, h,
                       state, yn, rtol, atol, n, c->d_red);
  }
  MAG_HIP(c, hipGetLastError());
  double en = 0.0;
  if ((rc = host_max(c, nb, &en))) return rc;
  if (failed(stages_status(c))) {
    *dt = 0.5 * h;
    return MAG_OK;
  }
  if (en <= 1.0) {
    MAG_HIP(c, hipMemcpyAsync(state, yn, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    std::swap(c->rk_k1, c->rk_k4);
    *t = *t + h;
    c->fsal_valid = true;
    c->fsal_state = state;
    c->fsal_t = *t;
    const double fac = en == 0.0 ? 5.0 : std::min(5.0, std::max(0.2, 0.8 * std::pow(en, -1.0 / 3.0)));
    *dt = h * fac;
    *accepted = 1;
  } else {
    const double fac = std::max(0.2, 0.8 * std::pow(en, -1.0 / 3.0));
    *dt = h * fac;
  }
  return MAG_OK;
}

static int launch_lincomb(mag_ctx *c, double *out, double a, const double *x, double b, const double *y,
                          long long n) {
  ProfScope ps(c, K_RK);
  hipLaunchKernelGGL(lincomb_k, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, out, a, x, b, y, n);
  MAG_HIP(c, hipGetLastError());
  return MAG_OK;
}

int mag_step_fixed(mag_ctx *c, double *state, double t, double dt) {
  CHECK_CTX(c);
  int rc = ready(c);
  if (rc) return rc;
  if (!state) return set_error(c, MAG_E_ARG, "NULL argument");
  if (!(dt > 0) || !std::isfinite(t)) return set_error(c, MAG_E_ARG, "need dt > 0 and a finite t");
  if ((rc = ensure_rk(c))) return rc;
  c->fsal_valid = false;
  double *k1 = rk_buf(c, 0), *k2 = rk_buf(c, 1), *k3 = rk_buf(c, 2), *yt = rk_buf(c, 4);
  const double h = dt;
  if ((rc = stage_rhs(c, state, t, k1))) return rc;
  if ((rc = launch_axpy(c, yt, state, k1, nullptr, nullptr, 1.0, 0, 0, 1, kA21 * h))) return rc;
  if ((rc = stage_rhs(c, yt, t + kRkC2 * h, k2))) return rc;
  if ((rc = launch_axpy(c, yt, state, k2, nullptr, nullptr, 1.0, 0, 0, 1, kA32 * h))) return rc;
  if ((rc = stage_rhs(c, yt, t + kRkC3 * h, k3))) return rc;
  if ((rc = launch_axpy(c, yt, state, k1, k2, k3, kB1, kB2, kB3, 3, h))) return rc;
  if (c->async_pending) {
    // the stages' status before the state is overwritten
    MAG_HIP(c, hipStreamSynchronize(c->stream));
    if ((rc = stages_status(c))) return rc;
  }
  return launch_lincomb(c, state, 1.0, yt, 0.0, nullptr, state_len(c));
}

// Transpose of mag_step_fixed at (state, t, dt): with y2 = y + h/2 k1 and
// y3 = y + 3h/4 k2 recomputed,
//   k3_bar = 4h/9 yb,  y3_bar = J(y3)^T k3_bar,
//   k2_bar = h/3 yb + 3h/4 y3_bar,  y2_bar = J(y2)^T k2_bar,
//   k1_bar = 2h/9 yb + h/2 y2_bar,  y1_bar = J(y)^T k1_bar,
//   y_bar = yb + y3_bar + y2_bar + y1_bar,
// and the jc-map cotangents of the three stages are added to jc_bar.
int mag_step_vjp(mag_ctx *c, const double *state, double t, double dt, const double *ybar_new, double *ybar,
                 double *jc_bar) {
  CHECK_CTX(c);
  int rc = ready(c);
  if (rc) return rc;
  if (!state || !ybar_new || !ybar) return set_error(c, MAG_E_ARG, "NULL argument");
  if (ybar == ybar_new || ybar == state) return set_error(c, MAG_E_ARG, "ybar must not alias ybar_new or state");
  if (!(dt > 0) || !std::isfinite(t)) return set_error(c, MAG_E_ARG, "need dt > 0 and a finite t");
  if ((rc = ensure_rk(c))) return rc;
  c->fsal_valid = false;
  const long long n = state_len(c), nj = c->nnode;
  double *A = rk_buf(c, 0), *Y2 = rk_buf(c, 1), *Y3 = rk_buf(c, 2), *D = rk_buf(c, 3), *E = rk_buf(c, 4);
  const double h = dt;
  int st;
  // forward stages
  if ((st = rhs_impl(c, state, t, A, nullptr))) return st;
  if ((rc = launch_axpy(c, Y2, state, A, nullptr, nullptr, 1.0, 0, 0, 1, kA21 * h))) return rc;
  if ((st = rhs_impl(c, Y2, t + kRkC2 * h, A, nullptr))) return st;
  if ((rc = launch_axpy(c, Y3, state, A, nullptr, nullptr, 1.0, 0, 0, 1, kA32 * h))) return rc;
  // reverse
  if ((rc = launch_lincomb(c, ybar, 1.0, ybar_new, 0.0, nullptr, n))) return rc;
  if ((rc = launch_lincomb(c, A, kB3 * h, ybar_new, 0.0, nullptr, n))) return rc;
  if ((st = rhs_vjp_impl(c, Y3, t + kRkC3 * h, A, D, jc_bar ? E : nullptr))) return st;
  if ((rc = launch_lincomb(c, ybar, 1.0, ybar, 1.0, D, n))) return rc;
  if (jc_bar && (rc = launch_lincomb(c, jc_bar, 1.0, jc_bar, 1.0, E, nj))) return rc;
  if ((rc = launch_lincomb(c, A, kB2 * h, ybar_new, kA32 * h, D, n))) return rc;
  if ((st = rhs_vjp_impl(c, Y2, t + kRkC2 * h, A, D, jc_bar ? E : nullptr))) return st;
  if ((rc = launch_lincomb(c, ybar, 1.0, ybar, 1.0, D, n))) return rc;
  if (jc_bar && (rc = launch_lincomb(c, jc_bar, 1.0, jc_bar, 1.0, E, nj))) return rc;
  if ((rc = launch_lincomb(c, A, kB1 * h, ybar_new, kA21 * h, D, n))) return rc;
  if ((st = rhs_vjp_impl(c, state, t, A, D, jc_bar ? E : nullptr))) return st;
  if ((rc = launch_lincomb(c, ybar, 1.0, ybar, 1.0, D, n))) return rc;
  if (jc_bar && (rc = launch_lincomb(c, jc_bar, 1.0, jc_bar, 1.0, E, nj))) return rc;
  return MAG_OK;
}

int mag_observe_vjp(mag_ctx *c, const double *hz_bar, double *state_bar) {
  CHECK_CTX(c);
  int rc = ready(c);
  if (rc) return rc;
  if (!hz_bar || !state_bar) return set_error(c, MAG_E_ARG, "NULL argument");
  if (c->dim == 3) return set_error(c, MAG_E_STATE, "3D observation transpose not available");
  return film_hz_transpose(c, hz_bar, state_bar);
}

int mag_step(mag_ctx *c, double *state, double *t, double *dt, double rtol, double atol, int *accepted) {
  CHECK_CTX(c);
  int rc = ready(c);
  if (rc) return rc;
  if (!state || !t || !dt || !accepted) return set_error(c, MAG_E_ARG, "NULL argument");
  if (!(*dt > 0) || !std::isfinite(*t) || !(rtol > 0) || !(atol > 0))
    return set_error(c, MAG_E_ARG, "need dt > 0, rtol > 0, atol > 0");
  return step_impl(c, state, t, dt, rtol, atol, accepted);
}

int mag_integrate(mag_ctx *c, double *state, double t0, double t1, double rtol, double atol, double *obs,
                  int obs_cap, int *n_steps) {
  CHECK_CTX(c);
  int rc = ready(c);
  if (rc) return rc;
  if (!state || !n_steps) return set_error(c, MAG_E_ARG, "NULL argument");
  if (!(t1 > t0) || !(rtol > 0) || !(atol > 0)) return set_error(c, MAG_E_ARG, "need t1 > t0, rtol > 0, atol > 0");
  if ((rc = ensure_rk(c))) return rc;
  *n_steps = 0;
  const long long n = state_len(c);
  double t = t0;
  int it0 = 0;
  rc = rhs_impl(c, state, t, rk_buf(c, c->rk_k1), &it0);
  if (rc) return rc;
  c->fsal_valid = true;
  c->fsal_state = state;
  c->fsal_t = t;
  if ((rc = ensure_red(c, n))) return rc;
  const int nb = (int)((n + 255) / 256);
  {
    ProfScope ps(c, K_RK);
    hipLaunchKernelGGL(rk_ratio_k, dim3(nb), dim3(256), 0, c->stream, rk_buf(c, c->rk_k1), state, atol / rtol, n, c->d_red);
  }
  MAG_HIP(c, hipGetLastError());
  double mx = 0.0;
  if ((rc = host_max(c, nb, &mx))) return rc;
  const double rh = mx / (0.8 * std::cbrt(rtol));
  double h = 0.1 * std::fabs(t1 - t0);
  if (rh * h > 1.0) h = 1.0 / rh;
  long long attempts = 0;
  while (t < t1 && attempts < 10000000LL) {
    if (1.1 * h >= t1 - t) h = t1 - t;
    if (h <= 16.0 * 2.220446049250313e-16 * std::max(std::fabs(t), 1.0))
      return set_error(c, MAG_STEP_UNDERFLOW, "step size underflow at t = %g", t);
    int acc = 0;
    const double hstep = h;
    rc = step_impl(c, state, &t, &h, rtol, atol, &acc);
    ++attempts;
    if (rc) return rc;
    if (acc) {
      if (obs && *n_steps < obs_cap) {
        double m[3] = {0, 0, 0};
        rc = c->dim == 3 ? bulk_observe(c, state, t, nullptr, nullptr, m) : film_observe(c, state, t, nullptr, nullptr, m);
        if (rc) return rc;
        double *o = obs + 6LL * (*n_steps);
        o[0] = t;
        o[1] = hstep;
        o[2] = m[0];
        o[3] = m[1];
        o[4] = m[2];
        o[5] = (double)c->last_iters;
      }
      ++*n_steps;
    }
  }
  return MAG_OK;
}

// ---------------------------------------------------------------- device-driven integration
static int ensure_capture(mag_ctx *c) {
  if (!c->d_sc) MAG_HIP(c, hipMalloc(&c->d_sc, sizeof(StepCtl)));
  if (!c->h_sc) MAG_HIP(c, hipHostMalloc(&c->h_sc, sizeof(StepCtl), hipHostMallocCoherent));
  // a stream of the library's own (default priority): capture needs one that
  // is not the legacy default stream
  if (!c->cap_stream) MAG_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  for (hipEvent_t &e : c->cap_ev)
    if (!e) MAG_HIP(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return MAG_OK;
}

// One step attempt of the device-driven integration, enqueued on c->stream:
// the three stage right-hand sides (film, fixed inner count), the stage sums,
// the error norm, accept / dt and the commit.  Buffers: k1..k4 = 0..3,
// y_stage = 4, y_new = 5.
static int enqueue_attempt(mag_ctx *c, double *state) {
  const long long n = state_len(c);
  double *k1 = rk_buf(c, 0), *k2 = rk_buf(c, 1), *k3 = rk_buf(c, 2), *k4 = rk_buf(c, 3);
  double *yt = rk_buf(c, 4), *yn = rk_buf(c, 5);
  const unsigned nbe = (unsigned)((n + 255) / 256);
  FieldZ f;
  f.kind = c->fkind;
  f.dz = c->fdir[2];
  f.amp = c->famp;
  f.omega = c->fomega;
  f.rate = c->frate;
  IterState base{};
  base.fixed = c->fixed_iters;
  base.inv_nout = c->nout > 0 ? 1.0 / (double)c->nout : 0.0;
  struct Stage {
    double cs;
    const double *k0, *k1, *k2;
    double w0, w1, w2, hfac;
    int nk;
    double *y, *k;
  };
  const Stage st[3] = {{kRkC2, k1, k1, k1, 1.0, 0.0, 0.0, kA21, 1, yt, k2},
                       {kRkC3, k2, k2, k2, 1.0, 0.0, 0.0, kA32, 1, yt, k3},
                       {1.0, k1, k2, k3, kB1, kB2, kB3, 1.0, 3, yn, k4}};
  for (int s = 0; s < 3; ++s) {
    {
      ProfScope ps(c, K_RK);
      hipLaunchKernelGGL(rk_axpy_sc_k, dim3(nbe), dim3(256), 0, c->stream, st[s].y, state, st[s].k0, st[s].k1,
                         st[s].k2, st[s].w0, st[s].w1, st[s].w2, st[s].nk, st[s].hfac, c->d_sc, n);
      hipLaunchKernelGGL(stage_init_k, dim3(1), dim3(64), 0, c->stream, c->d_it, c->h_it, c->d_sc, f, st[s].cs, base,
                         c->tol, s > 0 ? 1 : 0);
    }
    if (int rc = film_rhs_enqueue(c, st[s].y, st[s].k)) return rc;
  }
  ProfScope ps(c, K_RK);
  const unsigned nbr = (unsigned)((n + 256 * kErrNpt - 1) / (256 * kErrNpt));
  hipLaunchKernelGGL(rk_errnorm_sc_k, dim3(nbr), dim3(256), 0, c->stream, k1, k2, k3, k4, kE1, kE2, kE3, kE4, state,
                     yn, c->d_sc, n, c->d_red);
  hipLaunchKernelGGL(step_accept_k, dim3(1), dim3(256), 0, c->stream, c->d_sc, c->h_sc, c->d_red, (int)nbr, c->d_it);
  hipLaunchKernelGGL(step_commit_k, dim3(nbe), dim3(256), 0, c->stream, state, yn, k1, k4, c->d_sc, n);
  MAG_HIP(c, hipGetLastError());
  return MAG_OK;
}

int mag_integrate_captured(mag_ctx *c, double *state, double t0, double t1, double rtol, double atol, int chunk,
                           long long max_attempts, int *n_accepted, int *n_rejected, double *t_reached) {
  CHECK_CTX(c);
  int rc = ready(c);
  if (rc) return rc;
  if (!state) return set_error(c, MAG_E_ARG, "NULL argument");
  if (!(t1 > t0) || !(rtol > 0) || !(atol > 0) || !std::isfinite(t0) || !std::isfinite(t1))
    return set_error(c, MAG_E_ARG, "need finite t1 > t0, rtol > 0, atol > 0");
  if (chunk < 1 || chunk > 256 || max_attempts < 1) return set_error(c, MAG_E_ARG, "need 1 <= chunk <= 256, max_attempts >= 1");
  if (c->dim != 2 || c->fixed_iters <= 0)
    return set_error(c, MAG_E_STATE, "the captured integration needs a film and a fixed inner count");
  const long long n = state_len(c);
  if ((rc = ensure_rk(c)) || (rc = ensure_red(c, n)) || (rc = ensure_capture(c))) return rc;
  // k1 = f(state, t0) and the initial step as in mag_integrate (host driven, synchronising)
  c->rk_k1 = 0;
  c->rk_k4 = 3;
  c->fsal_valid = false;
  int it0 = 0;
  rc = rhs_impl(c, state, t0, rk_buf(c, 0), &it0);
  if (rc) return rc;
  const int nb = (int)((n + 255) / 256);
  {
    ProfScope ps(c, K_RK);
    hipLaunchKernelGGL(rk_ratio_k, dim3(nb), dim3(256), 0, c->stream, rk_buf(c, 0), state, atol / rtol, n, c->d_red);
  }
  MAG_HIP(c, hipGetLastError());
  double mx = 0.0;
  if ((rc = host_max(c, nb, &mx))) return rc;
  const double rh = mx / (0.8 * std::cbrt(rtol));
  double h = 0.1 * std::fabs(t1 - t0);
  if (rh * h > 1.0) h = 1.0 / rh;
  if (1.1 * h >= t1 - t0) h = t1 - t0;
  StepCtl sc{};
  sc.t = t0;
  sc.h = h;
  sc.t_end = t1;
  sc.rtol = rtol;
  sc.atol = atol;
  *c->h_sc = sc;
  MAG_HIP(c, hipMemcpyAsync(c->d_sc, c->h_sc, sizeof(StepCtl), hipMemcpyHostToDevice, c->stream));
  MAG_HIP(c, hipStreamSynchronize(c->stream));
  // the graph of `chunk` attempts, captured on the library's stream (rebuilt
  // when the state buffer, the chunk or any set-up changed)
  if (!c->cap_exec || c->cap_state != state || c->cap_chunk != chunk || c->cap_gen != c->gen) {
    release_capture(c);
    hipStream_t user = c->stream;
    const bool prof = c->prof_on, dbg = c->debug_sync;
    c->prof_on = false;
    c->debug_sync = false;   // no synchronisation while capturing
    c->stream = c->cap_stream;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    int rc2 = MAG_OK;
    if (e == hipSuccess) {
      for (int a = 0; a < chunk && rc2 == MAG_OK; ++a) rc2 = enqueue_attempt(c, state);
      e = hipStreamEndCapture(c->cap_stream, &g);
    }
    c->stream = user;
    c->prof_on = prof;
    c->debug_sync = dbg;
    if (rc2 != MAG_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc2;
    }
    if (e != hipSuccess) return hip_check(c, e, "stream capture of the step graph");
    e = hipGraphInstantiate(&c->cap_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->cap_exec = nullptr;
      return hip_check(c, e, "hipGraphInstantiate");
    }
    c->cap_state = state;
    c->cap_chunk = chunk;
    c->cap_gen = c->gen;
  }
  // replays on the library's stream, ordered after the caller's stream
  MAG_HIP(c, hipEventRecord(c->cap_ev[0], c->stream));
  MAG_HIP(c, hipStreamWaitEvent(c->cap_stream, c->cap_ev[0], 0));
  long long launched = 0;
  while (launched < max_attempts) {
    MAG_HIP(c, hipGraphLaunch(c->cap_exec, c->cap_stream));
    launched += chunk;
    MAG_HIP(c, hipStreamSynchronize(c->cap_stream));
    if (c->h_sc->finished) break;
  }
  MAG_HIP(c, hipEventRecord(c->cap_ev[1], c->cap_stream));
  MAG_HIP(c, hipStreamWaitEvent(c->stream, c->cap_ev[1], 0));
  const StepCtl v = *c->h_sc;
  if (n_accepted) *n_accepted = v.accepted;
  if (n_rejected) *n_rejected = v.rejected;
  if (t_reached) *t_reached = v.t;
  c->stat_rhs += 3LL * (v.accepted + v.rejected);
  c->stat_inner += 3LL * (v.accepted + v.rejected) * c->fixed_iters;
  // buffer 0 holds f(state, t) for the next step (first same as last)
  c->fsal_valid = true;
  c->fsal_state = state;
  c->fsal_t = v.t;
  c->warm_valid = true;
  c->async_pending = false;
  if (c->h_it->fail) {
    // the last attempt failed a stage and was rejected; the state is the last accepted one
    c->warm_valid = false;
  }
  if (v.status == MAG_STEP_UNDERFLOW) return set_error(c, MAG_STEP_UNDERFLOW, "step size underflow at t = %g", v.t);
  if (!v.finished) return set_error(c, MAG_NOT_CONVERGED, "t = %g not reached after %lld attempts", v.t, launched);
  return MAG_OK;
}

int mag_observe(mag_ctx *c, const double *state, double t, double *hz, double *j, double *m) {
  CHECK_CTX(c);
  int rc = ready(c);
  if (rc) return rc;
  if (!state || !m) return set_error(c, MAG_E_ARG, "state/m is NULL");
  return c->dim == 3 ? bulk_observe(c, state, t, hz, j, m) : film_observe(c, state, t, hz, j, m);
}

int mag_rhs_vjp(mag_ctx *c, const double *state, double t, const double *out_bar, double *state_bar,
                double *jc_bar) {
  CHECK_CTX(c);
  int rc = ready(c);
  if (rc) return rc;
  if (!state || !out_bar || !state_bar) return set_error(c, MAG_E_ARG, "NULL argument");
  return rhs_vjp_impl(c, state, t, out_bar, state_bar, jc_bar);
}

int mag_stats(mag_ctx *c, int reset, long long *n_rhs, long long *n_inner) {
  if (!c) return MAG_E_ARG;
  if (n_rhs) *n_rhs = c->stat_rhs;
  if (n_inner) *n_inner = c->stat_inner;
  if (reset) c->stat_rhs = c->stat_inner = 0;
  return MAG_OK;
}

int mag_prof_enable(mag_ctx *c, int on) {
  if (!c) return MAG_E_ARG;
  (void)hipStreamSynchronize(c->stream);
  prof_clear(c);
  if (on < 0 || on >= 2 + K_COUNT) return set_error(c, MAG_E_ARG, "prof mode must be 0, 1 or 2 + kernel id");
  c->prof_on = on != 0;
  c->prof_only = on >= 2 ? on - 2 : -1;
  return MAG_OK;
}

int mag_prof_read(mag_ctx *c, int id, int *count, double *total_ms) {
  if (!c || id < 0 || id >= K_COUNT || !count || !total_ms) return MAG_E_ARG;
  MAG_HIP(c, hipStreamSynchronize(c->stream));
  int cnt = 0;
  double tot = 0.0;
  for (auto &r : c->prof) {
    if (r.kid != id) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      tot += ms;
      ++cnt;
    }
  }
  *count = cnt;
  *total_ms = tot;
  return MAG_OK;
}

const char *mag_prof_kernel_name(int id) { return (id >= 0 && id < K_COUNT) ? mag::kNames[id] : nullptr; }

}  // extern "C"
