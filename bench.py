"""Benchmark: right-hand-side evaluations per second of the FFT-based method.

The headline metric is quoted on the bulk 256^3 configuration (128^3-cell
cube, tilted field, log-normal jc, n = 50).  That configuration is not run:
the 3D path is held off the GPU (its first GPU run faulted and the cause has
not been shown), so `value` is null and the line says why.

What is measured is the thin-film method on its largest workload, film-2048:
1024^2-cell films in a 2048^2 periodic grid on [-2,2]^2, ring (hole filled by
a normal conductor, rho_out = 500) and slotted square masks, log-normal jc
(s = 0.2, correlation length 8 cells), n = 30, h_e = 0.8 sin(1.25 t); mixed
precision (FP32 FFTs, multipliers and power law, FP64 state and sums) and
FP64, in two forms:

* fixed count: one right-hand-side evaluation = stencil pass + 4 inner
  iterations (10)-(12) from h_e on a Bean-like snapshot already resident in
  HBM, so that both precisions do the same work, with the same relaxation as
  the converged form (`film_2048_fixed4`);
* converged: the right-hand sides of an adaptive BS23 window (stop test of
  Sec. 2.3, warm start from the previous call as in Sec. 2.2) on a state
  reached by integrating from the virgin state, with the relaxation below
  2 / mu_max of the staggered iteration on this grid (`film_2048_converged`,
  with the mean inner iteration count I).

Prints one JSON line.  The throughput comes from a loop without any
instrumentation; per-kernel durations come from a further loop of the same
run in which the library attaches HIP start/stop events to the dispatch of
each transform kernel (hipExtLaunchKernelGGL, so no marker packets are timed
with the kernel): the breakdown, and the mean duration of the dominant kernel
(the roofline figure).  Further figures: the VJP of the same right-hand side
(adjoint/forward time ratio), adaptive BS23 step attempts on the same grid
(bs23_step_ms, and its ratio to three right-hand sides enqueued back to
back), and the error of the mixed form per result on a 256^2 trajectory.
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "RHS evals/s at 256^3 padded grid (mixed vs FP64) + adjoint/forward time ratio"
UNMEASURED = ("bulk-256 (128^3-cell cube in a 256^3 grid, n=50, tilted field, log-normal jc) not run: the 3D "
              "path is held off the GPU after an unexplained GPU fault in its first run")
# Relaxation of (12) for the 2048^2 films: the staggered iteration converges
# only for lambda * mu_max < 2, mu_max being the largest eigenvalue of
# (P K2 P)(P K1 P) on the free space (3.83 for the ring, about 5 for the slot
# at 2048^2, by power iteration on the oracle's operators).
LAMBDA_2048 = {"ring": 0.4, "slot": 0.33}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mask", default="ring", choices=["ring", "slot"], help="mask of the headline line")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--quick", action="store_true", help="headline mask and one precision only")
    ap.add_argument("--quick-prec", default="mixed", choices=["mixed", "fp64", "final64"],
                    help="the precision of a --quick run (profiling of one form)")
    ap.add_argument("--t", type=float, default=0.6, help="snapshot time")
    ap.add_argument("--iters", type=int, default=4, help="inner iterations per right-hand side")
    ap.add_argument("--window", type=int, default=20, help="timed BS23 attempts of the converged line")
    ap.add_argument("--only-hole", action="store_true",
                    help="only the 768x512 film with a hole (Sec. 2.3, Fig. 3), e.g. for a kernel trace")
    ap.add_argument("--copy-check", action="store_true",
                    help="also run a plain 64 MiB read + 64 MiB write kernel 3 times (counter calibration)")
    return ap.parse_args()


def film_inputs(mask, t_snap):
    """Material, jc map and Bean-like snapshot of the film-2048 workload."""
    from paper_1801_04869_amd import workloads as W
    wl = W.workload("film-2048-" + mask)
    nx, ny = wl["n"]
    Lx, Ly = wl["L"]
    if mask == "ring":
        mat = W.film_ring(nx, ny, Lx, Ly, 0.5, 1.0)
    else:
        mat = W.film_slot(nx, ny, Lx, Ly, 1.0, 8)
    jc = W.lognormal_jc((ny, nx), wl["jc"]["s"], wl["jc"]["ell"], wl["jc"]["seed"])
    g = W.film_snapshot(mat, 2 * Lx / nx, delta=0.15, seed=wl["jc"]["seed"])
    return wl, mat, jc, g


def free_nodes(mat):
    """Free-space nodes of a film material: a node is inside when the four
    cells around it are film."""
    F = mat != 0
    inside = F & np.roll(F, 1, axis=1) & np.roll(F, 1, axis=0) & np.roll(np.roll(F, 1, axis=0), 1, axis=1)
    return int(F.size - inside.sum())


def alg_bytes(kernel, n, kx, ny, prec, iters, n_out, has_jc=True):
    """Algorithmic HBM bytes per launch of each kernel of a fixed-count
    right-hand side (every input read once, every output written once; n
    nodes, n_out of them in free space, kx*ny half-spectrum entries, `iters`
    inner iterations), averaged over that kernel's launches in one call."""
    sc = 16 if prec == "fp64" else 8      # complex
    sr = 8 if prec == "fp64" else 4       # iterate, weights
    ns = kx * ny
    K = iters
    table = {
        # g (double), material and jc around inside nodes; flags; H out
        "film_stencil": (8 + 1 + (sr if has_jc else 0)) * (n - n_out) + n + sr * n,
        # H, flags, w1 in; H out on free space; spectrum out
        "film_rows_fwd_h": 2 * sr * n + n + sr * n_out + sc * ns,
        # 2K launches, the last one takes only the stop decision
        "film_cols": (2 * K - 1) * 2 * sc * ns / (2 * K),
        # spectrum in and out, w2; the last of the K launches writes dh/dt (double)
        "film_rows_inv_g": 2 * sc * ns + sr * n + 8 * n / K,
        # K - 1 launches: spectrum in and out, w1, H in, H out on free space
        "film_rows_inv_upd": 2 * sc * ns + 2 * sr * n + sr * n_out,
    }
    v = table.get(kernel)
    return int(round(v)) if v is not None else None


def sources_hash():
    """First 16 hex digits of the SHA-256 of the film kernel sources."""
    import hashlib
    h = hashlib.sha256()
    for f in ("film.hip", "fft.h", "kern_common.h"):
        with open(os.path.join(ROOT, "paper_1801_04869_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel, prec):
    """HBM bytes per launch from the committed rocprofv3 counter summaries
    (a line `traffic <kernel> <prec> bytes_per_launch=<B> sources_sha256_16=<H>`
    in a file under profiles/), or None if there is none for this kernel or the
    kernel sources changed since."""
    import glob
    import re
    pat = re.compile(r"traffic %s %s bytes_per_launch=(\d+) sources_sha256_16=([0-9a-f]+)" % (kernel, prec))
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        m = pat.search(open(path).read())
        if m:
            return int(m.group(1)) if m.group(2) == sources_hash() else None
    return None


def make_ctx(prec, wl, mat, jc, fixed=0, lam=0.7, max_inner=200, deriv="staggered"):
    import torch
    from paper_1801_04869_amd import api
    nx, ny = wl["n"]
    ctx = api.Context(2, {"mixed": api.MIXED, "fp64": api.FP64, "final64": api.MIXED_FINAL64}[prec])
    ctx.set_grid(nx, ny, 1, *wl["L"])
    if deriv == "spectral":
        ctx.set_derivatives(api.SPECTRAL)
    ctx.set_domain(torch.from_numpy(mat).cuda())
    ctx.set_params(torch.from_numpy(jc).cuda(), 1.0, wl["nexp"], 1.0, wl["rho_out"])
    ctx.set_solver(lam, 2e-4, max_inner, fixed)
    f = wl["field"]
    ctx.set_field(f["kind"], f["dir"], f["amp"], f["omega"], f["rate"])
    return ctx


def run_gpu(prec, wl, mat, jc, g, steps, warmup, t, fixed=0, lam=0.7):
    """Loops of `steps` right-hand sides on the same snapshot: the timed loop
    without any instrumentation (the throughput), the same calls enqueued
    back to back, and one with HIP events on every launch (the per-kernel
    breakdown, and the mean duration of the dominant kernel for the
    roofline), then the VJP.
    Every call restarts the inner iteration from h_e (no warm start), so with a
    fixed inner count every call does the same work."""
    import torch
    ctx = make_ctx(prec, wl, mat, jc, fixed, lam=lam)
    state = torch.from_numpy(g).cuda()
    out = torch.empty_like(state)

    def loop(n):
        its = []
        for _ in range(n):
            ctx.reset_warm_start()
            st, it = ctx.rhs(state, t, out)
            assert st == 0, ctx.last_error()
            its.append(it)
        return its

    loop(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = loop(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the same calls enqueued back to back (fixed count, no per-call wait)
    t1 = time.perf_counter()
    for _ in range(steps):
        ctx.reset_warm_start()
        ctx.rhs(state, t, out, wait=False)
    ctx.rhs_status()
    torch.cuda.synchronize()
    dt_stream = time.perf_counter() - t1
    # per-kernel durations: each transform kernel is launched with start and
    # stop events attached to its own dispatch (hipExtLaunchKernelGGL)
    ctx.prof_enable(True)
    loop(steps)
    prof_all = ctx.prof_read()
    ctx.prof_enable(False)
    dominant = max((k for k in prof_all if alg_bytes(k, 1, 1, 1, prec, 4, 1)), key=lambda k: prof_all[k][1])
    prof_dom = {dominant: prof_all[dominant]}
    # VJP of the same right-hand side (same fixed count), timed like the forward
    ybar = torch.ones_like(state)
    gbar = torch.empty_like(state)
    jcbar = torch.empty_like(state)
    for _ in range(warmup):
        assert ctx.rhs_vjp(state, t, ybar, gbar, jcbar) == 0, ctx.last_error()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps):
        assert ctx.rhs_vjp(state, t, ybar, gbar, jcbar) == 0, ctx.last_error()
    torch.cuda.synchronize()
    dt_vjp = time.perf_counter() - t2
    # adaptive BS23 step attempts (mag_step, same fixed count) from the virgin
    # state g = 0 at t = 0, where every stage stays finite: three right-hand
    # sides enqueued without host waits, the stage sums, the error norm and
    # one host synchronisation per attempt
    y = torch.zeros_like(state)
    ts, hs = 0.0, 1e-7
    ctx.reset_warm_start()
    for _ in range(warmup):
        ts, hs, _ = ctx.step(y, ts, hs)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    n_acc = 0
    for _ in range(steps):
        ts, hs, acc = ctx.step(y, ts, hs)
        n_acc += acc
    torch.cuda.synchronize()
    dt_step = time.perf_counter() - t3
    # the same attempts with the step control on the device, replayed from a
    # captured graph of 16 attempts (the first call captures and instantiates)
    yc = torch.zeros_like(state)
    ctx.integrate_captured(yc, 0.0, 1.0, chunk=16, max_attempts=16)
    yc.zero_()
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    na, nr, _ = ctx.integrate_captured(yc, 0.0, 1.0, chunk=16, max_attempts=2 * 16)
    torch.cuda.synchronize()
    dt_cap = time.perf_counter() - t4
    res = dict(value=steps / dt, ms_per_step=1e3 * dt / steps, inner_iters=float(np.mean(iters)), prof=prof_all,
               dominant=dominant, prof_dom=prof_dom[dominant], out=out.cpu().numpy(),
               vjp_ms=1e3 * dt_vjp / steps, value_stream=steps / dt_stream, step_ms=1e3 * dt_step / steps,
               step_accepted=n_acc, step_finite=bool(torch.isfinite(y).all()),
               captured_step_ms=1e3 * dt_cap / (na + nr), captured_attempts=(na, nr))
    ctx.close()
    return res


def gradient_run(prec, wl, mat, jc, g_snap, t_snap, lam, iters, n_steps=32, every=16):
    """The h_z misfit gradient with respect to the per-cell jc map along a
    trajectory (checkpointed reverse driver, autograd.trajectory): the
    accepted step sizes of an adaptive run from the Bean-like snapshot are
    replayed from the same start (fixed inner count, every right-hand side
    from h_e), with a checkpoint every `every` steps; the loss is
    1/2 sum (h_z - 0)^2 dx dy at the last step.  Times the forward trajectory
    and the backward pass.  (From the snapshot the power law is active in the
    whole film, so the steps are short but the gradient is not zero, as it
    would be from g = 0, where |j| << jc makes rho(|j|) vanish.)"""
    import torch
    from paper_1801_04869_amd import autograd as ag
    ctx = make_ctx(prec, wl, mat, jc, iters, lam=lam)
    nx, ny = wl["n"]
    y = torch.from_numpy(g_snap).cuda()
    t, h, steps, attempts = t_snap, 1e-15, [], 0
    while len(steps) < n_steps:
        t1, h1, acc = ctx.step(y, t, h)
        if acc:
            steps.append(h)
        t, h = t1, h1
        attempts += 1
        assert attempts < 20 * n_steps, "adaptive run keeps rejecting"
    g0 = torch.from_numpy(g_snap).cuda()
    dA = (2 * wl["L"][0] / nx) * (2 * wl["L"][1] / ny)
    for rep in range(2):   # the first pass is a warm-up
        jc_t = torch.from_numpy(jc).cuda().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        (yl,) = ag.trajectory(ctx, g0, jc_t, t_snap, steps, [n_steps - 1], every=every)
        hz = ag.hz(ctx, yl, t_snap + sum(steps))
        loss = 0.5 * (hz * hz).sum() * dA
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    g = jc_t.grad
    ctx.close()
    return dict(steps=n_steps, checkpoint_every=every, t_span=sum(steps), forward_ms=round(1e3 * (t1 - t0), 2),
                backward_ms=round(1e3 * (t2 - t1), 2), backward_over_forward=round((t2 - t1) / (t1 - t0), 3),
                grad_finite=bool(torch.isfinite(g).all()), grad_norm=float(torch.linalg.norm(g)))


def observe_time(prec, wl, mat, jc, g, t, reps=20):
    """Mean time of mag_observe (h_z by the |k|/2 transform of g, j on the
    edges, the moment) on the snapshot, in ms."""
    import torch
    ctx = make_ctx(prec, wl, mat, jc, 4)
    state = torch.from_numpy(g).cuda()
    for _ in range(3):
        ctx.observe(state, t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.observe(state, t)   # returns the moment on the host: synchronises
    dt = time.perf_counter() - t0
    ctx.close()
    return round(1e3 * dt / reps, 4)


def spectral_run(prec, wl, mat, jc, g, steps, warmup, t, fixed, lam):
    """The fixed-count loop of run_gpu with the spectral form of Sec. 2.2
    (fields on the nodes, filtered Fourier derivatives): RHS/s without
    instrumentation, then the per-kernel breakdown from a loop with events
    on every dispatch."""
    import torch
    ctx = make_ctx(prec, wl, mat, jc, fixed, lam=lam, deriv="spectral")
    state = torch.from_numpy(g).cuda()
    out = torch.empty_like(state)

    def loop(n):
        for _ in range(n):
            ctx.reset_warm_start()
            st, it = ctx.rhs(state, t, out)
            assert st == 0, ctx.last_error()

    loop(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loop(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.prof_enable(True)
    loop(steps)
    prof = ctx.prof_read()
    ctx.prof_enable(False)
    # the VJP of the same right-hand side (the transposed spectral passes)
    ybar = torch.ones_like(state)
    gbar, jcbar = torch.empty_like(state), torch.empty_like(state)
    for _ in range(warmup):
        assert ctx.rhs_vjp(state, t, ybar, gbar, jcbar) == 0, ctx.last_error()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps):
        assert ctx.rhs_vjp(state, t, ybar, gbar, jcbar) == 0, ctx.last_error()
    torch.cuda.synchronize()
    dt_vjp = time.perf_counter() - t2
    ctx.close()
    per_rhs = {k: dict(launches_per_rhs=round(c / steps, 2), us_per_rhs=round(1e3 * ms / steps, 2),
                       avg_us=round(1e3 * ms / c, 2)) for k, (c, ms) in prof.items()}
    return dict(value=round(steps / dt, 3), unit="RHS evals/s", ms_per_step=round(1e3 * dt / steps, 4),
                adjoint_forward_ratio=round(dt_vjp / dt, 3), kernels=per_rhs)


def hole_film_lines(a):
    """RHS/s on the film of Sec. 2.3, Fig. 3: fixed count on a Bean-like
    snapshot and converged right-hand sides of an adaptive window from the
    virgin state, both film forms, mixed and FP64."""
    import torch
    from paper_1801_04869_amd import workloads as W
    wl = W.workload("film-768x512-hole")
    nx, ny = wl["n"]
    Lx, Ly = wl["L"]
    h = wl["hole"]
    mat = W.film_rect_hole(nx, ny, Lx, Ly, h["ax"], h["ay"], h["cx"], h["cy"], h["r"])
    jc = np.ones((ny, nx))
    g = W.film_snapshot(mat, 2 * Lx / nx, delta=0.15, seed=1806)
    out = dict(workload="film-768x512-hole: rectangle |x| <= 1.5, |y| <= 1 with the hole (x-0.5)^2 + (y-0.25)^2 "
                        "<= 0.25 filled by a normal conductor, 768x512 grid on |x| <= 2.25, |y| <= 1.5, n = 50, "
                        "rho_out = 500, h_e = t, uniform jc, lambda %g; fixed: %d inner iterations on a Bean-like "
                        "snapshot at t = 0.3; converged: adaptive BS23 window from g = 0" % (wl["lam"], a.iters))
    for form in ("staggered", "spectral"):
        for prec in ("mixed", "fp64"):
            ctx = make_ctx(prec, wl, mat, jc, a.iters, lam=wl["lam"], deriv=form)
            state = torch.from_numpy(g).cuda()
            o = torch.empty_like(state)
            for _ in range(a.warmup):
                ctx.reset_warm_start()
                ctx.rhs(state, 0.3, o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(a.steps):
                ctx.reset_warm_start()
                st, _ = ctx.rhs(state, 0.3, o)
                assert st == 0, ctx.last_error()
            torch.cuda.synchronize()
            fixed = a.steps / (time.perf_counter() - t0)
            ctx.close()
            conv = converged_window(prec, wl, mat, jc, wl["lam"], a.warmup, a.window, deriv=form)
            out["%s-%s" % (form, prec)] = dict(fixed_rhs_per_s=round(fixed, 1), converged=conv)
            print("[bench] film-768x512-hole %s %s: fixed %d %.1f RHS/s, converged %.1f RHS/s (I = %.2f)" %
                  (form, prec, a.iters, fixed, conv["value"], conv["mean_inner_iters"]), file=sys.stderr, flush=True)
    return out


def paper_runs():
    """The paper's timed whole runs in its own discretisation (the spectral
    form, FP64, adaptive BS23 with rtol 1e-3 / atol 1e-6, the stop test of
    Sec. 2.3): the disk of Table 1 (radius 1 in [-2, 2]^2, n = 1000,
    rho_out = 1, h_e = t to 0.5) at 128^2, 256^2 and 512^2, and the film
    with a hole of Sec. 2.3, Fig. 3 to t = 0.4: wall time, steps, right-hand
    sides.  The deviations from the Bean solution are checked by the GPU
    tests (tests/test_gpu_paper_runs.py), not here.  The paper's figures
    (Matlab on one CPU) are context, not targets."""
    import torch
    from paper_1801_04869_amd import api
    from paper_1801_04869_amd import workloads as W

    def run(mat, n, L, nexp, rho_out, lam, prec, t_end):
        c = api.Context(2, prec)
        c.set_grid(n[0], n[1], 1, *L)
        c.set_derivatives(api.SPECTRAL)
        c.set_domain(torch.from_numpy(mat).cuda())
        c.set_params(None, 1.0, nexp, 1.0, rho_out)
        c.set_solver(lam, 2e-4, 100, 0)
        c.set_field(api.RAMP, (0.0, 0.0, 1.0), 1.0, 1.0, 1.0)
        g = torch.zeros((n[1], n[0]), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps, _ = c.integrate(g, 0.0, t_end, 1e-3, 1e-6)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        n_rhs, n_inner = c.stats()
        _, j, (_, _, mz) = c.observe(g, t_end)
        c.close()
        return g, j.cpu().numpy(), dict(wall_s=round(wall, 3), steps=steps, rhs=n_rhs,
                                        mean_inner_iters=round(n_inner / max(n_rhs, 1), 2), m_z=mz)

    out = dict(form="spectral (Sec. 2.2), FP64 unless named, BS23 rtol 1e-3 atol 1e-6, stop test 2e-4",
               paper_hardware="Matlab R2017a on one Intel Core i5-2400 (context only)")
    table1 = {}
    for N, lam, pmin in ((128, 0.7, 0.2), (256, 0.7, 2.0), (512, 0.5, 49.0)):
        mat = W.film_disk(N, N, 2.0, 2.0, 1.0)
        g, j, r = run(mat, (N, N), (2.0, 2.0), 1000.0, 1.0, lam, api.FP64, 0.5)
        r.update(lambda_=lam, paper_wall_min=pmin)
        table1["disk-%d" % N] = r
        print("[bench] Table 1 disk %d^2: %.2f s, %d steps (paper %.1f min)" % (N, r["wall_s"], r["steps"], pmin),
              file=sys.stderr, flush=True)
    out["table1_disk"] = table1
    # the rectangle of Sec. 2.3, Fig. 2 (the paper gives no time for it)
    g, j, r = run(W.film_rect(1024, 256, 4.0, 1.0, 3.2, 0.5), (1024, 256), (4.0, 1.0), 1000.0, 1.0, 0.4,
                  api.FP64, 0.5)
    r.update(lambda_=0.4)
    out["strip_1024x256"] = r
    print("[bench] strip 1024x256 to h_e = 0.5: %.2f s, %d steps" % (r["wall_s"], r["steps"]), file=sys.stderr,
          flush=True)
    wl = W.workload("film-768x512-hole")
    h = wl["hole"]
    mat = W.film_rect_hole(*wl["n"], *wl["L"], h["ax"], h["ay"], h["cx"], h["cy"], h["r"])
    hole = {}
    states = {}
    for name, prec in (("fp64", api.FP64), ("mixed", api.MIXED), ("final64", api.MIXED_FINAL64)):
        g, j, r = run(mat, wl["n"], wl["L"], wl["nexp"], wl["rho_out"], wl["lam"], prec, 0.4)
        states[name] = g.cpu().numpy()
        r.update(lambda_=wl["lam"], paper_wall_min=63.0)
        hole[name] = r
        print("[bench] hole film 768x512 to t = 0.4, %s: %.2f s, %d steps (paper 63 min)" %
              (name, r["wall_s"], r["steps"]), file=sys.stderr, flush=True)
    for name in ("mixed", "final64"):
        hole["%s_vs_fp64_g_rel_l2" % name] = float(np.linalg.norm(states[name] - states["fp64"]) /
                                                  np.linalg.norm(states["fp64"]))
    out["hole_film_768x512_t04"] = hole
    return out


def converged_window(prec, wl, mat, jc, lam, warm_attempts, attempts, deriv="staggered"):
    """Right-hand sides of an adaptive BS23 run with the stop test: from the
    virgin state g = 0 at t = 0, `warm_attempts` step attempts (untimed) bring
    the film to a state reached by integration; the next `attempts` attempts
    are timed.  Every right-hand side is warm-started from the previous one's
    free-space solution (Sec. 2.2).  Returns RHS/s (right-hand sides counted by
    the library, stage sums and step control included in the time) and the
    mean inner iteration count."""
    import torch
    ctx = make_ctx(prec, wl, mat, jc, 0, lam=lam, max_inner=200, deriv=deriv)
    y = torch.zeros((wl["n"][1], wl["n"][0]), dtype=torch.float64, device="cuda")
    ts, hs = 0.0, 1e-7
    for _ in range(warm_attempts):
        ts, hs, _ = ctx.step(y, ts, hs)
    torch.cuda.synchronize()
    ctx.stats(reset=True)
    t0 = time.perf_counter()
    n_acc = 0
    for _ in range(attempts):
        ts, hs, acc = ctx.step(y, ts, hs)
        n_acc += acc
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_rhs, n_inner = ctx.stats()
    finite = bool(torch.isfinite(y).all())
    ctx.close()
    return dict(value=round(n_rhs / dt, 3), unit="RHS evals/s", rhs=n_rhs, mean_inner_iters=round(n_inner / n_rhs, 3),
                ms_per_rhs=round(1e3 * dt / n_rhs, 4), lambda_=lam, attempts=attempts, accepted=n_acc,
                t_end=ts, state_finite=finite)


ACC_N, ACC_T_END = 256, 0.005


def step_grid(ctx, state0, t, t_end):
    """Accepted (t, dt) of an adaptive BS23 run (rtol 1e-3, atol 1e-6) of
    `ctx` from state0 at t to t_end."""
    y = state0.clone()
    grid, dt = [], 1e-6
    while t < t_end:
        t1, dt1, acc = ctx.step(y, t, dt)
        if acc:
            grid.append((t, dt))   # the step taken is exactly the dt passed in
        t, dt = t1, dt1
        assert len(grid) < 5000, "too many steps"
    return grid


def trajectory(ctx, state0, grid):
    """Per-result accuracy input: BS23 steps on a given time grid (no error
    control, so both precisions take the same steps), then the observables at
    the end: (g, h_z, j, m) on the host."""
    import torch
    y = state0.clone()
    for t, dt in grid:
        assert ctx.step_fixed(y, t, dt) == 0, ctx.last_error()
    t, dt = grid[-1]
    hz, j, m = ctx.observe(y, t + dt)
    torch.cuda.synchronize()
    return y.cpu().numpy(), hz.cpu().numpy(), j.cpu().numpy(), np.array(m)


def per_result_error(mixed, fp64):
    """Relative L2 difference of each result of the mixed form from the FP64
    form after the same steps."""
    names = ("g", "hz", "j", "m")
    return {k: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
            for k, a, b in zip(names, mixed, fp64)}


def _oracle_rhs_times(mask, t, iters, reps):
    """Child-process body of the CPU baseline: the oracle's right-hand side of
    the film-2048 workload, `reps` times; prints the durations as JSON."""
    from oracle import film
    from oracle.field import AppliedField
    wl, mat, jc, g = film_inputs(mask, t)
    f = wl["field"]
    nx, ny = wl["n"]
    prob = film.FilmProblem(nx, ny, *wl["L"], mat, jc_cell=jc, n=wl["nexp"], rho_out=wl["rho_out"], lam=0.7,
                            tol=2e-4, max_inner=iters, fixed_iters=iters,
                            field=AppliedField(f["kind"], f["dir"], f["amp"], f["omega"], f["rate"]))
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        film.rhs(prob, g, t)
        times.append(time.perf_counter() - t0)
    print(json.dumps(times), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(mask, t, iters):
    """The oracle as it stands (NumPy FP64, pocketfft): the median of 3
    right-hand sides of the same workload at the same fixed inner count as the
    GPU line, in a child process pinned to core 0 with one thread per
    numerical library."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               NUMEXPR_NUM_THREADS="1", HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")
    cmd = [sys.executable, os.path.abspath(__file__), "--oracle-child", mask, repr(t), str(iters), "3"]
    pinned = True
    try:
        r = subprocess.run(["taskset", "-c", "0"] + cmd, capture_output=True, text=True, env=env, timeout=600)
    except FileNotFoundError:
        pinned = False
        r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=600)
    if r.returncode != 0:
        return dict(value=None, unit="RHS evals/s", cores=1, kind="oracle", error=r.stderr[-500:])
    times = json.loads(r.stdout.strip().splitlines()[-1])
    med = float(np.median(times))
    return dict(value=round(1.0 / med, 5), unit="RHS evals/s", cores=1, kind="oracle",
                sample="3 right-hand sides (%d inner iterations each) of the NumPy FP64 oracle on the same "
                       "2048^2 snapshot, median %.2f s; %s, OMP/BLAS threads 1" %
                       (iters, med, "pinned to core 0 (taskset -c 0)" if pinned else "not pinned (no taskset)"))


def kernel_table(prof, n, kx, ny, prec, iters, n_out):
    rows = {}
    for k, (cnt, ms) in prof.items():
        ab = alg_bytes(k, n, kx, ny, prec, iters, n_out)
        avg = ms / cnt * 1e-3
        rows[k] = dict(launches=cnt, avg_us=round(avg * 1e6, 2),
                       GBps=round(ab / avg / 1e9, 1) if ab else None)
    return rows


def accuracy(wl, deriv="staggered"):
    """Error of the two mixed forms per result: a ring film of the workload's
    structure at ACC_N^2 (same field, law, rho_out and jc statistics)
    integrated from the virgin state to ACC_T_END by the adaptive FP64 form
    with the converged inner iteration; the accepted time grid is replayed
    in every precision (each right-hand side started from h_e, so the replay
    repeats the run) and g, h_z, j, m at the end are compared with the FP64
    replay, as is one right-hand side at the end state."""
    import torch
    from paper_1801_04869_amd import workloads as W
    Lx, Ly = wl["L"]
    w = dict(wl, n=(ACC_N, ACC_N))
    mat = W.film_ring(ACC_N, ACC_N, Lx, Ly, 0.5, 1.0)
    jc = W.lognormal_jc((ACC_N, ACC_N), wl["jc"]["s"], wl["jc"]["ell"], wl["jc"]["seed"])
    state = torch.zeros((ACC_N, ACC_N), dtype=torch.float64, device="cuda")
    forms = ("mixed", "final64")
    ctx = {p: make_ctx(p, w, mat, jc, 0, deriv=deriv) for p in ("fp64",) + forms}
    for c in ctx.values():
        c.set_warm_start(False)
    grid = step_grid(ctx["fp64"], state, 0.0, ACC_T_END)
    res = {p: trajectory(c, state, grid) for p, c in ctx.items()}
    out = {p: per_result_error(res[p], res["fp64"]) for p in forms}
    t_end = grid[-1][0] + grid[-1][1]
    y = torch.from_numpy(res["fp64"][0]).cuda()
    o = {p: torch.empty_like(y) for p in ctx}
    for p, c in ctx.items():
        c.rhs(y, t_end, o[p])
        c.close()
    out["rhs_at_end"] = {p: (torch.linalg.norm(o[p] - o["fp64"]) / torch.linalg.norm(o["fp64"])).item()
                         for p in forms}
    out["after"] = ("%d^2 ring film (workload structure, %s form) from the virgin state, %d adaptive BS23 steps "
                    "to t = %.4g, converged inner iteration" % (ACC_N, deriv, len(grid), t_end))
    return out


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--oracle-child":
        _oracle_rhs_times(sys.argv[2], float(sys.argv[3]), int(sys.argv[4]), int(sys.argv[5]))
        return
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only; the multi-GPU layout is a design note, not a measured path.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.only_hole:
        print(json.dumps(dict(film_768x512_hole=hole_film_lines(a))), flush=True)
        return
    masks = [a.mask] if a.quick else [a.mask] + [m for m in ("ring", "slot") if m != a.mask]
    precs = [a.quick_prec] if a.quick else ["mixed", "fp64", "final64"]
    hp = precs[0]   # precision of the roofline and kernel-table lines
    res = {}
    inputs = {}
    for mask in masks:
        inputs[mask] = film_inputs(mask, a.t)
        wl, mat, jc, g = inputs[mask]
        for prec in precs:
            r = run_gpu(prec, wl, mat, jc, g, a.steps, a.warmup, a.t, fixed=a.iters, lam=LAMBDA_2048[mask])
            res[(mask, prec)] = r
            print("[bench] film-2048-%s %s fixed %d: %.1f RHS/s, %.3f ms/RHS" %
                  (mask, prec, a.iters, r["value"], r["ms_per_step"]), file=sys.stderr, flush=True)
    conv = {}
    for mask in masks:
        wl, mat, jc, g = inputs[mask]
        for prec in precs:
            c = converged_window(prec, wl, mat, jc, LAMBDA_2048[mask], a.warmup, a.window)
            conv["%s-%s" % (mask, prec)] = c
            print("[bench] film-2048-%s %s converged: %.1f RHS/s, I = %.2f, %d/%d accepted, t = %.3g" %
                  (mask, prec, c["value"], c["mean_inner_iters"], c["accepted"], c["attempts"], c["t_end"]),
                  file=sys.stderr, flush=True)
    wl, mat, jc, g = inputs[a.mask]
    nx, ny = wl["n"]
    n, kx = nx * ny, nx // 2 + 1
    n_out = free_nodes(mat)
    m = res[(a.mask, hp)]
    kern = m["dominant"]
    cnt, tot = m["prof_dom"]
    avg_s = tot / cnt * 1e-3
    ab = alg_bytes(kern, n, kx, ny, hp, a.iters, n_out)
    achieved = ab / avg_s / 1e9
    film_workload = ("film-2048-%s: 1024^2-cell %s film in a 2048^2 periodic grid, n=30, log-normal jc (s=0.2, "
                     "l=8 cells), h_e=0.8 sin(1.25 t), Bean-like snapshot at t=%g; %d inner iterations per RHS"
                     % (a.mask, a.mask, a.t, a.iters))
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=recorded_traffic(kern, hp), kernel=kern,
                bytes_per_launch=ab, avg_launch_us=round(avg_s * 1e6, 2), workload=film_workload + ", " + hp)
    fixed_lines = {}
    for (mask, prec), r in res.items():
        fixed_lines["%s-%s" % (mask, prec)] = dict(value=round(r["value"], 3), unit="RHS evals/s",
                                                   ms_per_step=round(r["ms_per_step"], 4),
                                                   inner_iters=round(r["inner_iters"], 3),
                                                   value_enqueued_back_to_back=round(r["value_stream"], 3),
                                                   adjoint_forward_ratio=round(r["vjp_ms"] / r["ms_per_step"], 3))
    line = dict(metric=METRIC, value=None, unit="RHS evals/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
                ms_per_step=None, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32+f64",
                data="synthetic",
                config=dict(workload=UNMEASURED, measured="film-2048 (thin-film method), below"),
                roofline=roof)
    line["film_2048_fixed%d" % a.iters] = dict(workload=film_workload, lines=fixed_lines)
    line["film_2048_fixed%d" % a.iters]["kernels_" + hp] = kernel_table(m["prof"], n, kx, ny, hp, a.iters, n_out)
    line["film_2048_converged"] = dict(
        workload="film-2048 ring/slot, adaptive BS23 (rtol 1e-3, atol 1e-6) from g = 0 at t = 0: %d untimed "
                 "attempts, then %d timed attempts; stop test 2e-4 max(|dh_e/dt|, 1), warm start, lambda %s"
                 % (a.warmup, a.window, LAMBDA_2048), lines=conv)
    if (a.mask, "fp64") in res and hp == "mixed":
        f64 = res[(a.mask, "fp64")]
        line["mixed_over_fp64_fixed"] = round(m["value"] / f64["value"], 3)
        d = m["out"] - f64["out"]
        line["mixed_vs_fp64_rel_l2"] = float(np.linalg.norm(d) / max(np.linalg.norm(f64["out"]), 1e-300))
        line["mixed_vs_fp64_per_result"] = accuracy(wl)
        # the form whose results stay within 1e-4 of FP64 along the trajectory
        # (final evaluation of (11) in double) against FP64, same workloads
        f6 = res.get((a.mask, "final64"))
        if f6 is not None:
            line["final64_over_fp64_fixed"] = round(f6["value"] / f64["value"], 3)
        line["over_fp64_converged"] = {
            "%s-%s" % (mask, p): round(conv["%s-%s" % (mask, p)]["value"] / conv["%s-fp64" % mask]["value"], 3)
            for mask in masks for p in ("mixed", "final64") if "%s-%s" % (mask, p) in conv}
        line["film_2048_fixed%d" % a.iters]["kernels_fp64"] = kernel_table(f64["prof"], n, kx, ny, "fp64", a.iters,
                                                                           n_out)
    # the paper's own discretisation (spectral form) on the headline mask
    sp_lines = {}
    for prec in precs:
        r = spectral_run(prec, wl, mat, jc, g, a.steps, a.warmup, a.t, a.iters, LAMBDA_2048[a.mask])
        r["over_staggered"] = round(r["value"] / res[(a.mask, prec)]["value"], 3)
        sp_lines[prec] = r
        print("[bench] film-2048-%s spectral %s fixed %d: %.1f RHS/s" % (a.mask, prec, a.iters, r["value"]),
              file=sys.stderr, flush=True)
    sp_conv = {}
    for prec in precs[:1] if a.quick else ("mixed", "fp64"):
        c = converged_window(prec, wl, mat, jc, LAMBDA_2048[a.mask], a.warmup, a.window, deriv="spectral")
        sp_conv[prec] = c
        print("[bench] film-2048-%s spectral %s converged: %.1f RHS/s, I = %.2f" %
              (a.mask, prec, c["value"], c["mean_inner_iters"]), file=sys.stderr, flush=True)
    line["film_2048_spectral"] = dict(
        workload=film_workload + "; spectral form of Sec. 2.2 (j, e and dh_z/dt on the nodes from filtered "
                                 "Fourier derivatives, sigma = sqrt(dx^2 + dy^2))",
        fixed=sp_lines, converged=sp_conv)
    # in this form MAG_MIXED itself stays within 1e-4 of FP64 per result along
    # a converged trajectory (tests/test_gpu_mixed_accuracy.py): its speed-up at
    # equal accuracy
    if "mixed" in sp_lines and "fp64" in sp_lines:
        line["film_2048_spectral"]["mixed_over_fp64_fixed"] = round(sp_lines["mixed"]["value"] /
                                                                    sp_lines["fp64"]["value"], 3)
    if "mixed" in sp_conv and "fp64" in sp_conv:
        line["film_2048_spectral"]["mixed_over_fp64_converged"] = round(sp_conv["mixed"]["value"] /
                                                                        sp_conv["fp64"]["value"], 3)
    if not a.quick:
        line["film_2048_spectral"]["mixed_vs_fp64_per_result"] = accuracy(wl, deriv="spectral")
    # the film with a circular hole of Sec. 2.3, Fig. 3 (768 x 512, radix-12 row transforms)
    if not a.quick:
        line["film_768x512_hole"] = hole_film_lines(a)
        line["paper_runs"] = paper_runs()
    line["adjoint_forward_ratio_film"] = round(m["vjp_ms"] / m["ms_per_step"], 3)
    line["bs23_step_ms"] = round(m["step_ms"], 4)
    line["bs23_step_over_3_rhs"] = round(m["step_ms"] * m["value_stream"] / 3e3, 3)
    line["bs23_steps"] = "%d attempts from g = 0 at t = 0, %d accepted, state finite: %s" % (
        a.steps, m["step_accepted"], m["step_finite"])
    line["bs23_captured_step_ms"] = round(m["captured_step_ms"], 4)
    line["bs23_captured_step_over_3_rhs"] = round(m["captured_step_ms"] * m["value_stream"] / 3e3, 3)
    line["bs23_captured"] = ("step control on the device, 32 attempts (%d accepted) from g = 0 at t = 0 replayed "
                             "from a captured graph of 16 attempts (one host synchronisation per replay); the "
                             "first right-hand side and step size on the host" % m["captured_attempts"][0])
    if not a.quick:
        line["observe_ms"] = {p: observe_time(p, wl, mat, jc, g, a.t) for p in ("mixed", "fp64")}
        gr = gradient_run("mixed", wl, mat, jc, g, a.t, LAMBDA_2048[a.mask], a.iters)
        gr["workload"] = ("film-2048-%s, mixed, %d inner iterations: h_z misfit gradient with respect to the jc map "
                          "over %d replayed adaptive steps from the Bean-like snapshot at t = %g, checkpoints "
                          "every %d steps" % (a.mask, a.iters, gr["steps"], a.t, gr["checkpoint_every"]))
        line["film_2048_gradient"] = gr
        print("[bench] film-2048-%s gradient: forward %.1f ms, backward %.1f ms (%.2fx), finite %s" %
              (a.mask, gr["forward_ms"], gr["backward_ms"], gr["backward_over_forward"], gr["grad_finite"]),
              file=sys.stderr, flush=True)
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(a.mask, a.t, a.iters)
        line["cpu_baseline"]["workload"] = film_workload
    line["host"] = dict(cpu=cpu_model(), cpu_count=os.cpu_count(), numpy=np.__version__)
    if a.copy_check:
        src = torch.ones(16 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        line["copy_check"] = "3 x elementwise kernel reading 64 MiB and writing 64 MiB"
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
