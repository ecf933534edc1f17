/*
 * magfft -- FFT-based magnetization of type-II superconductors on one MI355X.
 *
 * C ABI of the method-of-lines right-hand side of Prigozhin & Sokolovsky,
 * "FFT-based solution of 2D and 3D magnetization problems in type-II
 * superconductivity":
 *   dim 2 (thin film, Sec. 2): state g = stream function on nodes, eq. (2);
 *         f(g, t) is the discretised iteration (11)-(12) with dh_z/dt in the
 *         film from eq. (9).
 *   dim 3 (bulk, Sec. 3):      state h = magnetic field on Yee-lattice edges;
 *         f(h, t) is Faraday's law (14) with the power law (13) in Omega plus
 *         iteration (18) with the Biot-Savart operator Phi of eq. (17).
 * Everything is in the paper's dimensionless units (Sec. 2.3 and eq. (19)).
 *
 * Discretisation shared by both dimensions:
 *   box D = [-L_a, L_a] per axis, periodic through the FFT (Sec. 2.2, 3.1);
 *   n_a nodes at -L_a + i d_a, d_a = 2 L_a / n_a; cell i spans nodes i..i+1.
 *   Arrays are row-major with x fastest: 2D [ny][nx], 3D [nz][ny][nx].
 *   Derivatives are staggered finite differences; the film current sits on
 *   edges, the bulk current j = curl h on faces (component c of h on the edge
 *   half-shifted along axis c, component c of j on the face normal to c).
 *   A node (2D) / edge (3D) is "inside" when all cells around it are
 *   non-vacuum; every other node/edge is free space, where the iteration
 *   determines the time derivative.
 *
 * Memory: every pointer argument marked "device" is caller-owned device memory
 * (e.g. a contiguous torch tensor); the library never frees it or keeps it
 * after the call returns.  The context owns all workspace (allocated by
 * mag_set_grid / mag_set_domain and the first mag_step) and frees it in
 * mag_destroy.  Pointers marked "host" are ordinary host memory.
 *
 * Streams: all device work is enqueued on the stream given to mag_create.
 * Calls that return host scalars synchronise that stream before returning.
 *
 * Errors: negative return codes are hard errors.  MAG_E_ARG and MAG_E_STATE
 * leave the context unchanged; MAG_E_HIP marks it unusable.  Positive codes
 * are numerical statuses.  mag_last_error returns a description of the most
 * recent failure.  A context is not thread-safe.
 *
 * Sizes: each n_a must be a power of two, 16 <= n_a <= 2048 (nz = 1 in 2D).
 */
#ifndef MAGFFT_H
#define MAGFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mag_ctx mag_ctx;

enum mag_status {
  MAG_OK = 0,
  MAG_NOT_CONVERGED = 1,   /* inner iteration did not reach its tolerance in max_inner steps */
  MAG_STEP_UNDERFLOW = 2,  /* integrator step fell below 16 eps |t| */
  MAG_E_ARG = -1,          /* invalid argument (size, pointer, value) */
  MAG_E_STATE = -2,        /* call out of order (e.g. rhs before set_domain) */
  MAG_E_HIP = -3,          /* HIP runtime error; the context must be destroyed */
  MAG_E_NOMEM = -4,        /* device allocation failed */
  MAG_E_NUMERIC = -5       /* non-finite value in the state or the result */
};

enum mag_precision {
  MAG_FP64 = 0,  /* everything in double precision */
  MAG_MIXED = 1, /* FFTs, Fourier multipliers and the power law in float; state,
                    time stepping, step control and all iteration sums in double */
  MAG_MIXED_FINAL64 = 2  /* films only: the iteration (11)-(12) as MAG_MIXED, then the
                    returned dg/dt evaluated once more by (11) in double from the
                    iterate the float iteration stopped at (FFTs, multiplier 2/|k|
                    and the free-space mean in double).  Observables and the VJP
                    are those of MAG_MIXED.  mag_create returns MAG_E_ARG for it
                    with dim = 3. */
};

enum mag_deriv_form {
  MAG_DERIV_STAGGERED = 0, /* films (default): j on cell edges by differences of g
                              (eq. (2)), e on the edges, (9) by differences back
                              to the nodes */
  MAG_DERIV_SPECTRAL = 1   /* films: every field on the nodes, each derivative the
                              filtered Fourier multiplier of Sec. 2.2 */
};

enum mag_field_kind {
  MAG_FIELD_RAMP = 0,   /* h_e(t) = rate * t * dir            (Sec. 2.3: h_e = t) */
  MAG_FIELD_SINE = 1,   /* h_e(t) = amp * sin(omega t) * dir  (Sec. 3.2 cube benchmark) */
  MAG_FIELD_ROTATE = 2  /* h_e(t) = amp * (cos omega t, sin omega t, 0) */
};

/* Create a context for dim = 2 (film) or 3 (bulk) with the given precision.
 * hip_stream: a hipStream_t (may be NULL for the default stream).
 * Errors: MAG_E_ARG for a bad dim/precision/out pointer. */
int mag_create(mag_ctx **out, int dim, int precision, void *hip_stream);

/* Free the context and everything it owns.  NULL is ignored. */
void mag_destroy(mag_ctx *ctx);

/* Uniform grid on D = [-Lx,Lx] x [-Ly,Ly] (x [-Lz,Lz]) with nx x ny (x nz)
 * nodes (Sec. 2.2 and 3.1).  nz must be 1 for dim 2.  Allocates the FFT and
 * iteration workspace.  Sizes: powers of two in [16, 2048]; a film may also
 * have nx or ny = 3 * 2^k in [48, 768] (the 768 x 512 film of Sec. 2.3,
 * Fig. 3), transformed with a radix-12 first stage.
 * Errors: MAG_E_ARG (other sizes, non-positive lengths), MAG_E_NOMEM; MAG_E_STATE for a 3D grid
 * in GPU builds: the 3D path is compiled but disabled there (held off the GPU
 * after an unexplained memory fault); only the CPU emulation build of the
 * sources enables it. */
int mag_set_grid(mag_ctx *ctx, int nx, int ny, int nz, double Lx, double Ly, double Lz);

/* Material per cell, device uint8 array [nz][ny][nx] (nz = 1 in 2D):
 * 0 free space, 1 superconductor (power law), 2 normal conductor with the
 * resistivity rho_out (a filled hole, Sec. 2.2; a cut layer, Sec. 3.1).
 * Copied; derives the inside/free-space classification and the pruning box.
 * Errors: MAG_E_STATE before set_grid; MAG_E_ARG for codes > 2 or an empty
 * sample. */
int mag_set_domain(mag_ctx *ctx, const uint8_t *material);

/* Power law (3)/(13): rho(|j|) = (e0 / jc)(|j| / jc)^(n-1) in superconducting
 * cells, rho_out in normal cells.  jc per cell = jc0 * jc_map[cell] (device
 * double array [nz][ny][nx], copied) or jc0 when jc_map is NULL; the jc of an
 * edge/face is the mean of its two cells.  Errors: MAG_E_ARG for n < 1,
 * jc0 <= 0, e0 <= 0, rho_out < 0, or a non-positive jc_map entry. */
int mag_set_params(mag_ctx *ctx, const double *jc_map, double jc0, double n, double e0,
                   double rho_out);

/* Inner-iteration control.  lambda: relaxation of (12) (film only; Sec. 2.2
 * uses 0.7).  inner_tol: stop when the mean free-space |gdot| (film, Sec. 2.3)
 * or mean free-space |dh^{i+1} - dh^i| (bulk, Sec. 3.1) is below
 * inner_tol * max(|dh_e/dt|, 1).  max_inner: iteration cap; exceeding it
 * returns MAG_NOT_CONVERGED.  fixed_iters > 0: run exactly that many
 * iterations without a stop test (used to compare implementations).
 * Defaults: 0.7, 2e-4 (film) / 1e-4 (bulk), 100, 0. */
int mag_set_solver(mag_ctx *ctx, double lambda, double inner_tol, int max_inner, int fixed_iters);

/* Uniform applied field, see enum mag_field_kind.  dir: host double[3]
 * (only the z component is used in 2D).  Default: ramp along z, rate 1. */
int mag_set_field(mag_ctx *ctx, int kind, const double dir[3], double amp, double omega,
                  double rate);

/* One right-hand-side evaluation out = f(state, t).
 * state, out: device double arrays of nx*ny (2D) or 3*nx*ny*nz (3D, component
 *   planes [3][nz][ny][nx]); out must not alias state.
 * n_inner (host, nullable): number of inner iterations used.
 * The free-space part of the previous call's result is the first guess
 * (warm start, Sec. 2.2); it is dropped after MAG_NOT_CONVERGED.
 * Returns MAG_OK, MAG_NOT_CONVERGED (out undefined) or an error.
 * With a fixed iteration count (mag_set_solver fixed_iters > 0, film) and
 * n_inner == NULL the call only enqueues the work and returns MAG_OK at once;
 * mag_rhs_status then waits and reports a non-finite result. */
int mag_rhs(mag_ctx *ctx, const double *state, double t, double *out, int *n_inner);

/* Wait for the context's stream; report MAG_E_NUMERIC if the last
 * asynchronous mag_rhs produced a non-finite residual (and drop the warm
 * start), MAG_OK otherwise.  n_inner (host, nullable): inner iterations of the
 * last right-hand side. */
int mag_rhs_status(mag_ctx *ctx, int *n_inner);

/* One adaptive Bogacki-Shampine 3(2) step attempt (the pair of Matlab's
 * ode23 used in Sec. 2.2) from (state, *t) with step *dt.
 * On acceptance state (device) and *t (host) advance and *accepted = 1; on
 * rejection both stay and *accepted = 0.  *dt (host) receives the next step
 * size either way.  Error norm max_i |err_i| / max(rtol max(|y_i|,|ynew_i|),
 * atol); step factor min(5, max(0.2, 0.8 err^(-1/3))) after acceptance,
 * max(0.2, 0.8 err^(-1/3)) after rejection, 1/2 when an inner iteration did
 * not converge or a stage value is not finite.  The first-same-as-last stage
 * is reused while state and *t are unchanged since the previous accepted
 * call.  With a fixed inner count (film) the stages after the first are
 * enqueued without host waits and the call synchronises once, for the error
 * norm; with the stop test each stage polls the host as mag_rhs does. */
int mag_step(mag_ctx *ctx, double *state, double *t, double *dt, double rtol, double atol,
             int *accepted);

/* Integrate from t0 to t1 with mag_step (first step 0.1 (t1 - t0) limited
 * by 0.8 rtol^(1/3) / max_i(|f_i| / max(|y_i|, atol / rtol)); the last step
 * lands on t1).  state: device, advanced in place.  obs (host, nullable):
 * room for obs_cap records of 6 doubles per accepted step:
 * t, dt, m_x, m_y, m_z, inner iterations of the step's last stage.
 * n_steps (host): accepted steps.  Returns MAG_STEP_UNDERFLOW if the step
 * collapses. */
int mag_integrate(mag_ctx *ctx, double *state, double t0, double t1, double rtol, double atol,
                  double *obs, int obs_cap, int *n_steps);

/* mag_integrate with the step control on the device (Sec. 2.2: the adaptive
 * Bogacki-Shampine pair of ode23 around the right-hand side), for a film
 * with a fixed inner count (mag_set_solver fixed_iters > 0; MAG_E_STATE
 * otherwise).  After the first right-hand side and the first step size (as
 * mag_integrate), t and dt live in device memory: each step attempt (three
 * stage right-hand sides, the stage sums, the error norm, accept / reject
 * with the controller of mag_step, the end-time clip and the commit of the
 * accepted state) is a fixed sequence of kernels with no host decision.
 * `chunk` attempts are captured once into a HIP graph on a stream of the
 * library's own (ordered after the context's stream by events) and the
 * graph is replayed until t1 is reached or max_attempts attempts have run,
 * with one host synchronisation per replay.  The instantiated graph is kept
 * and reused while the state buffer, the chunk and every set-up call stay
 * the same.  A stage whose residual turns non-finite rejects the attempt
 * with dt / 2 and the next attempt restarts its free-space iteration from
 * dh_e/dt.  state: device FP64, advanced in place (its last accepted value).
 * n_accepted, n_rejected, t_reached: host, nullable.  Returns MAG_OK when t1
 * is reached, MAG_STEP_UNDERFLOW if the step collapses, MAG_NOT_CONVERGED if
 * max_attempts ran out first.  1 <= chunk <= 256. */
int mag_integrate_captured(mag_ctx *ctx, double *state, double t0, double t1, double rtol, double atol,
                           int chunk, long long max_attempts, int *n_accepted, int *n_rejected,
                           double *t_reached);

/* Observables of a state (post-processing, Sec. 2.1 last formula):
 * 2D: hz (device, nx*ny, nodes) = h_e + F^{-1}[|k|/2 F(g)]; j (device,
 *     2*nx*ny: j_x on x-edges then j_y on y-edges, eq. (2); at the nodes in
 *     the spectral form of mag_set_derivatives); m[0..2] (host)
 *     = (0, 0, sum g dx dy).
 * 3D: hz (device, nx*ny*nz) = z component of h on z-edges; j (device,
 *     3*nx*ny*nz) = curl h on faces; m (host) = (1/2) sum r x j dV.
 * hz and j may be NULL. */
int mag_observe(mag_ctx *ctx, const double *state, double t, double *hz, double *j, double *m);

/* Vector-Jacobian product of mag_rhs at (state, t): state_bar = (df/dstate)^T
 * out_bar and jc_bar = (df/djc_map)^T out_bar (both device, same layouts as
 * state and jc_map; jc_bar may be NULL).  The free-space iteration is
 * differentiated as its converged fixed point (or, with fixed_iters, as
 * exactly that many iterations); the warm start is a constant.  Overwrites
 * state_bar and jc_bar. */
int mag_rhs_vjp(mag_ctx *ctx, const double *state, double t, const double *out_bar,
                double *state_bar, double *jc_bar);

/* Forget the warm start: the next mag_rhs starts from dh_e/dt. */
int mag_reset_warm_start(mag_ctx *ctx);

/* Discretisation of the film right-hand side (eqs. (2)-(4) in the form (9)),
 * films only (MAG_E_ARG for dim = 3 or another mode).
 * MAG_DERIV_STAGGERED (the default): differences on the staggered grid.
 * MAG_DERIV_SPECTRAL (Sec. 2.2): all fields live on the nodes and d/dx_a is
 * the multiplier i k_a exp(-|k|^2 sigma^2 / 2), the Nyquist wavenumber of
 * axis a set to zero.  j = (d_y g, -d_x g); e = rho(|j|) j, the power law (3)
 * at nodes whose four cells are superconducting (jc the mean of the four
 * cells) and rho_out at every other node; dh_z/dt = -(d_x e_y - d_y e_x) at
 * the film nodes.  sigma < 0 selects the width of Sec. 2.2, sqrt(dx^2 + dy^2),
 * for the grid in force at each call.  The update (12) stays unfiltered in
 * both forms.  mag_observe then returns j at the nodes (j_x, then j_y, each
 * nx*ny), and mag_rhs_vjp transposes this form (the filtered derivatives are
 * antisymmetric; the jc cotangent of a node goes to its four cells).
 * May be called before or after mag_set_grid; the spectral form holds three
 * more half spectra and two more node arrays on the device (allocated here or
 * by mag_set_grid, not by mag_rhs or mag_rhs_vjp).  Drops the warm start. */
int mag_set_derivatives(mag_ctx *ctx, int mode, double sigma);

/* on = 0: every right-hand side starts the free-space iteration from dh_e/dt
 * (no warm start), which makes f a function of (state, t) alone -- needed
 * when a trajectory is recomputed for gradients; on = 1 (default): warm
 * start from the previous call (Sec. 2.2). */
int mag_set_warm_start(mag_ctx *ctx, int on);

/* One Bogacki-Shampine step of exactly dt from (state, t), without error
 * control (replay of an accepted step): state (device) advances in place.
 * Returns MAG_NOT_CONVERGED if an inner iteration fails, MAG_E_NUMERIC if a
 * stage value is not finite; the state is unchanged in both cases.  With a
 * fixed inner count (film) the three stages are enqueued without host waits
 * and the call synchronises once, before the state is written. */
int mag_step_fixed(mag_ctx *ctx, double *state, double t, double dt);

/* Transpose of mag_step_fixed at (state, t, dt) with dt frozen: ybar
 * (device, overwritten) = (d state_new / d state)^T ybar_new; jc_bar (device
 * [nz][ny][nx], may be NULL) is ADDED the jc-map cotangent of the step.  The
 * stages are recomputed (three right-hand sides) and pulled back with
 * mag_rhs_vjp semantics.  ybar must not alias ybar_new or state. */
int mag_step_vjp(mag_ctx *ctx, const double *state, double t, double dt, const double *ybar_new,
                 double *ybar, double *jc_bar);

/* Transpose of the map state -> h_z of mag_observe (h_e excluded):
 * state_bar (device, overwritten) from hz_bar (device).  2D: the multiplier
 * |k|/2 (Sec. 2.1) applied to hz_bar.  3D: MAG_E_STATE. */
int mag_observe_vjp(mag_ctx *ctx, const double *hz_bar, double *state_bar);

/* Text of the most recent error or status (never NULL). */
const char *mag_last_error(const mag_ctx *ctx);

/* ---- instrumentation (timing of individual kernels, for benchmarks) ----
 * mag_prof_enable(ctx, 1) times every kernel launch on the context's stream:
 * the film transform and stencil kernels (one launch per record) through
 * HIP start/stop events attached to their own dispatch, the other records
 * through a pair of event records around their launches (which adds the
 * markers' own time); mag_prof_enable(ctx, 2 + id) times launches of kernel
 * `id` only (the events cost host time per launch); mag_prof_enable(ctx, 0)
 * stops and clears.
 * mag_prof_read sums the recorded durations of kernel `id` (synchronising the
 * stream): *count launches, *total_ms milliseconds.  Launches that found the
 * iteration already converged and returned at once are not recorded.
 * mag_prof_kernel_name(id) names kernel id (NULL past the last id). */
int mag_prof_enable(mag_ctx *ctx, int on);
int mag_prof_read(mag_ctx *ctx, int id, int *count, double *total_ms);
const char *mag_prof_kernel_name(int id);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the film
 * magnetic moment of mag_observe, m = (0, 0, sum of g dx dy) with
 * dx = 2 Lx / nx, dy = 2 Ly / ny, without a context and without allocating.
 * g: device FP64 stream function [ny][nx]; m: device, 3 doubles, written
 * (no host copy, no synchronisation); hip_stream: the stream to enqueue on
 * (NULL = the default stream).  Per-block partial sums live in a library
 * array of MAG_NOALLOC_MAX_PARTS doubles on each device (held until the
 * process ends), so nx * ny must not exceed MAG_NOALLOC_MAX_PARTS * 2048
 * nodes (MAG_E_ARG otherwise, nothing enqueued).  Every call on a device
 * uses the same array: calls that overlap on one device (other streams,
 * other threads) race and must be ordered by the caller.  The array's device
 * address is looked up by mag_create, or by the first call on a device.
 * Returns MAG_OK, MAG_E_ARG or MAG_E_HIP. */
#define MAG_NOALLOC_MAX_PARTS 8192
int mag_film_moment_noalloc(const double *g, int nx, int ny, double Lx, double Ly, double *m, void *hip_stream);

/* Counts of the work done since the last reset: *n_rhs right-hand sides
 * evaluated (mag_rhs and the stages of mag_step / mag_integrate /
 * mag_step_fixed) and *n_inner inner iterations (evaluations of (11) in 2D,
 * updates (18) in 3D) summed over them; a fixed count enqueued without a
 * host wait counts its fixed number.  reset != 0 zeroes the counts after
 * reading them.  Host pointers; either may be NULL.  Instrumentation for
 * reporting the mean inner iteration count, no GPU work. */
int mag_stats(mag_ctx *ctx, int reset, long long *n_rhs, long long *n_inner);

#ifdef __cplusplus
}
#endif
#endif /* MAGFFT_H */
