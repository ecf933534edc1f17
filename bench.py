"""Benchmark: right-hand-side evaluations per second of the thin-film method.

Workload film-2048: 1024^2-cell films in a 2048^2 periodic grid on [-2,2]^2,
ring (hole filled by a normal conductor, rho_out = 500) and slotted square
masks, log-normal jc (s = 0.2, correlation length 8 cells), n = 30,
h_e = 0.8 sin(1.25 t); mixed precision (FP32 FFTs, multipliers and power law,
FP64 state and sums) and FP64.  The bulk 256^3 configuration is not measured:
the 3D path is held off the GPU.

One "step" = one right-hand-side evaluation (stencil pass + a fixed count of
inner iterations (10)-(12), 4 by default, so that both precisions do the same
work) on a Bean-like snapshot already resident in HBM.  A fixed count is used
because on this snapshot, which is not a state reached by time integration,
the iteration with lambda = 0.7 does not reach the stop test at 2048^2.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mask", default="ring", choices=["ring", "slot"], help="mask of the headline line")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--quick", action="store_true", help="headline mask and mixed precision only")
    ap.add_argument("--t", type=float, default=0.6, help="snapshot time")
    ap.add_argument("--iters", type=int, default=4, help="inner iterations per right-hand side")
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


def make_ctx(prec, wl, mat, jc, fixed=0):
    import torch
    from paper_1801_04869_amd import api
    nx, ny = wl["n"]
    ctx = api.Context(2, api.MIXED if prec == "mixed" else api.FP64)
    ctx.set_grid(nx, ny, 1, *wl["L"])
    ctx.set_domain(torch.from_numpy(mat).cuda())
    ctx.set_params(torch.from_numpy(jc).cuda(), 1.0, wl["nexp"], 1.0, wl["rho_out"])
    ctx.set_solver(0.7, 2e-4, 200, fixed)
    f = wl["field"]
    ctx.set_field(f["kind"], f["dir"], f["amp"], f["omega"], f["rate"])
    return ctx


def run_gpu(prec, wl, mat, jc, g, steps, warmup, t, fixed=0):
    """Loops of `steps` right-hand sides on the same snapshot: the timed loop
    without any instrumentation (the throughput), the same calls enqueued
    back to back, and one with HIP events on every launch (the per-kernel
    breakdown, and the mean duration of the dominant kernel for the
    roofline), then the VJP.
    Every call restarts the inner iteration from h_e (no warm start), so with a
    fixed inner count every call does the same work."""
    import torch
    ctx = make_ctx(prec, wl, mat, jc, fixed)
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
    res = dict(value=steps / dt, ms_per_step=1e3 * dt / steps, inner_iters=float(np.mean(iters)), prof=prof_all,
               dominant=dominant, prof_dom=prof_dom[dominant], out=out.cpu().numpy(),
               vjp_ms=1e3 * dt_vjp / steps, value_stream=steps / dt_stream, step_ms=1e3 * dt_step / steps,
               step_accepted=n_acc, step_finite=bool(torch.isfinite(y).all()))
    ctx.close()
    return res


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


def cpu_baseline(wl, mat, jc, g, t, iters):
    """The oracle as it stands (NumPy FP64, pocketfft, single-threaded): the
    median of 3 right-hand sides of the same workload at the same fixed inner
    count as the GPU line."""
    from oracle import film
    from oracle.field import AppliedField
    f = wl["field"]
    nx, ny = wl["n"]
    prob = film.FilmProblem(nx, ny, *wl["L"], mat, jc_cell=jc, n=wl["nexp"], rho_out=wl["rho_out"], lam=0.7,
                            tol=2e-4, max_inner=iters, fixed_iters=iters,
                            field=AppliedField(f["kind"], f["dir"], f["amp"], f["omega"], f["rate"]))
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        film.rhs(prob, g, t)
        times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    return dict(value=round(1.0 / med, 5), unit="RHS evals/s", cores=1, kind="oracle",
                sample="3 right-hand sides (%d inner iterations each) of the NumPy FP64 oracle on the same "
                       "2048^2 snapshot, median %.2f s" % (iters, med))


def kernel_table(prof, n, kx, ny, prec, iters, n_out):
    rows = {}
    for k, (cnt, ms) in prof.items():
        ab = alg_bytes(k, n, kx, ny, prec, iters, n_out)
        avg = ms / cnt * 1e-3
        rows[k] = dict(launches=cnt, avg_us=round(avg * 1e6, 2),
                       GBps=round(ab / avg / 1e9, 1) if ab else None)
    return rows


def accuracy(wl):
    """Error of the mixed form per result: a ring film of the workload's
    structure at ACC_N^2 (same field, law, rho_out and jc statistics)
    integrated from the virgin state to ACC_T_END by the adaptive FP64 form
    with the converged inner iteration; the accepted time grid is replayed
    in both precisions (each right-hand side started from h_e, so the replay
    repeats the run) and g, h_z, j, m at the end are compared, as is one
    right-hand side at the end state."""
    import torch
    from paper_1801_04869_amd import workloads as W
    Lx, Ly = wl["L"]
    w = dict(wl, n=(ACC_N, ACC_N))
    mat = W.film_ring(ACC_N, ACC_N, Lx, Ly, 0.5, 1.0)
    jc = W.lognormal_jc((ACC_N, ACC_N), wl["jc"]["s"], wl["jc"]["ell"], wl["jc"]["seed"])
    state = torch.zeros((ACC_N, ACC_N), dtype=torch.float64, device="cuda")
    ctx = {p: make_ctx(p, w, mat, jc, 0) for p in ("fp64", "mixed")}
    for c in ctx.values():
        c.set_warm_start(False)
    grid = step_grid(ctx["fp64"], state, 0.0, ACC_T_END)
    res = {p: trajectory(c, state, grid) for p, c in ctx.items()}
    out = per_result_error(res["mixed"], res["fp64"])
    t_end = grid[-1][0] + grid[-1][1]
    y = torch.from_numpy(res["fp64"][0]).cuda()
    o = {p: torch.empty_like(y) for p in ctx}
    for p, c in ctx.items():
        c.rhs(y, t_end, o[p])
        c.close()
    out["rhs_at_end"] = (torch.linalg.norm(o["mixed"] - o["fp64"]) / torch.linalg.norm(o["fp64"])).item()
    out["after"] = ("%d^2 ring film (workload structure) from the virgin state, %d adaptive BS23 steps to "
                    "t = %.4g, converged inner iteration" % (ACC_N, len(grid), t_end))
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only; the multi-GPU layout is a design note, not a measured path.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    masks = [a.mask] if a.quick else [a.mask] + [m for m in ("ring", "slot") if m != a.mask]
    precs = ["mixed"] if a.quick else ["mixed", "fp64"]
    res = {}
    inputs = {}
    for mask in masks:
        inputs[mask] = film_inputs(mask, a.t)
        wl, mat, jc, g = inputs[mask]
        for prec in precs:
            r = run_gpu(prec, wl, mat, jc, g, a.steps, a.warmup, a.t, fixed=a.iters)
            res[(mask, prec)] = r
            print("[bench] film-2048-%s %s: %.1f RHS/s, %.3f ms/RHS, %.2f inner iterations" %
                  (mask, prec, r["value"], r["ms_per_step"], r["inner_iters"]), file=sys.stderr, flush=True)
    wl, mat, jc, g = inputs[a.mask]
    nx, ny = wl["n"]
    n, kx = nx * ny, nx // 2 + 1
    n_out = free_nodes(mat)
    m = res[(a.mask, "mixed")]
    kern = m["dominant"]
    cnt, tot = m["prof_dom"]
    avg_s = tot / cnt * 1e-3
    ab = alg_bytes(kern, n, kx, ny, "mixed", a.iters, n_out)
    achieved = ab / avg_s / 1e9
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=recorded_traffic(kern, "mixed"), kernel=kern,
                bytes_per_launch=ab, avg_launch_us=round(avg_s * 1e6, 2))
    line = dict(metric=METRIC, value=round(m["value"], 3), unit="RHS evals/s", n_gpus=1, steps=a.steps,
                warmup=a.warmup, ms_per_step=round(m["ms_per_step"], 4), higher_is_better=True, scaling="weak",
                vs_baseline=None, dtype="f32+f64", data="synthetic",
                config=dict(workload="film-2048-%s: 1024^2-cell %s film in a 2048^2 periodic grid, n=30, "
                                     "log-normal jc (s=0.2, l=8 cells), h_e=0.8 sin(1.25 t), Bean-like snapshot "
                                     "at t=%g; %d inner iterations per RHS" % (a.mask, a.mask, a.t, a.iters),
                            precision="mixed", inner_iters=a.iters,
                            bulk_256="not measured: 3D path held off the GPU"),
                inner_iters=round(m["inner_iters"], 3),
                value_enqueued_back_to_back=round(m["value_stream"], 3), roofline=roof,
                kernels_mixed=kernel_table(m["prof"], n, kx, ny, "mixed", a.iters, n_out))
    others = {}
    for (mask, prec), r in res.items():
        if (mask, prec) == (a.mask, "mixed"):
            continue
        others["%s-%s" % (mask, prec)] = dict(value=round(r["value"], 3), ms_per_step=round(r["ms_per_step"], 4),
                                              inner_iters=round(r["inner_iters"], 3),
                                              adjoint_forward_ratio=round(r["vjp_ms"] / r["ms_per_step"], 3))
    if others:
        line["other_lines"] = others
    if (a.mask, "fp64") in res:
        f64 = res[(a.mask, "fp64")]
        line["mixed_over_fp64"] = round(m["value"] / f64["value"], 3)
        # accuracy of the mixed form against the FP64 form on the same snapshot
        d = m["out"] - f64["out"]
        line["mixed_vs_fp64_rel_l2"] = float(np.linalg.norm(d) / max(np.linalg.norm(f64["out"]), 1e-300))
        line["mixed_vs_fp64_per_result"] = accuracy(wl)
        line["kernels_fp64"] = kernel_table(f64["prof"], n, kx, ny, "fp64", a.iters, n_out)
    line["adjoint_forward_ratio"] = round(m["vjp_ms"] / m["ms_per_step"], 3)
    line["bs23_step_ms"] = round(m["step_ms"], 4)
    line["bs23_step_over_3_rhs"] = round(m["step_ms"] * m["value_stream"] / 3e3, 3)
    line["bs23_steps"] = "%d attempts from g = 0 at t = 0, %d accepted, state finite: %s" % (
        a.steps, m["step_accepted"], m["step_finite"])
    line["adjoint_ms_per_rhs"] = round(m["vjp_ms"], 4)
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(wl, mat, jc, g, a.t, a.iters)
    line["host"] = dict(cpu=platform.processor() or platform.machine(), cpu_count=os.cpu_count(),
                        numpy=np.__version__)
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
