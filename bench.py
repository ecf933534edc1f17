"""Benchmark: right-hand-side evaluations per second of the bulk method on the
bulk-256 workload (128^3-cell cube in a 256^3 periodic grid, n = 50, field
ramp tilted 30 degrees from z, log-normal jc with s = 0.15 and correlation
length 6 cells), mixed precision and FP64, plus the adjoint/forward time
ratio when the adjoint is available.

One "step" = one right-hand-side evaluation (stencil pass + converged inner
iteration) on a Bean-like snapshot already resident in HBM.  Prints one JSON
line.  Per-kernel durations come from HIP events recorded around every launch
during the timed region (on the library's stream).
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="bulk-256")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--t", type=float, default=0.3, help="snapshot time")
    return ap.parse_args()


def bulk_inputs(name, t_snap):
    from paper_1801_04869_amd import workloads as W
    wl = W.workload(name)
    nx, ny, nz = wl["n"]
    Lx, Ly, Lz = wl["L"]
    mat = W.bulk_box(nx, ny, nz, Lx, Ly, Lz, *wl["half"])
    jc = None
    if "jc" in wl:
        jc = W.lognormal_jc((nz, ny, nx), wl["jc"]["s"], wl["jc"]["ell"], wl["jc"]["seed"])
    f = wl["field"]
    d = np.asarray(f["dir"], dtype=np.float64)
    if f["kind"] == 0:
        he = d * f["rate"] * t_snap
    elif f["kind"] == 1:
        he = d * f["amp"] * np.sin(f["omega"] * t_snap)
    else:
        he = f["amp"] * np.array([np.cos(f["omega"] * t_snap), np.sin(f["omega"] * t_snap), 0.0])
    h = W.bulk_snapshot(mat, 2 * Lx / nx, he, delta=0.2, seed=1804)
    return wl, mat, jc, h


def alg_bytes(kernel, c, prec):
    """Algorithmic HBM bytes per launch of each iteration kernel."""
    nx, ny, nz = c["n"]
    kx = nx // 2 + 1
    b0, b1 = c["box0"], c["box1"]
    bx, by, bz = (b1[a] - b0[a] + 1 for a in range(3))
    sc = 16 if prec == "fp64" else 8
    sr = 8 if prec == "fp64" else 4
    N = nx * ny * nz
    if kernel == "bulk_x_fwd":
        return 3 * by * bz * bx * sr + by * bz * bx + 3 * by * bz * kx * sc
    if kernel == "bulk_y_fwd":
        return 3 * kx * by * bz * sc + 3 * kx * ny * bz * sc
    if kernel == "bulk_z_phi":
        return 3 * kx * ny * bz * sc + 3 * kx * ny * nz * sc
    if kernel == "bulk_y_inv":
        return 2 * 3 * kx * ny * nz * sc
    if kernel == "bulk_x_inv":
        return 3 * kx * ny * nz * sc + N + 2 * 3 * N * sr
    return None


def box_of(mat):
    """Node box holding every inside face/edge (same rule as the library)."""
    f = mat != 0
    idx = np.nonzero(f)
    lo = [int(idx[2].min()), int(idx[1].min()), int(idx[0].min())]
    hi = [int(idx[2].max()), int(idx[1].max()), int(idx[0].max())]
    return lo, hi


def run_gpu(prec, wl, mat, jc, h, steps, warmup, t):
    import torch
    from paper_1801_04869_amd import api
    P = api.MIXED if prec == "mixed" else api.FP64
    nx, ny, nz = wl["n"]
    ctx = api.Context(3, P)
    ctx.set_grid(nx, ny, nz, *wl["L"])
    ctx.set_domain(torch.from_numpy(mat).cuda())
    ctx.set_params(None if jc is None else torch.from_numpy(jc).cuda(), 1.0, wl["nexp"], 1.0, 1.0)
    ctx.set_solver(0.7, 1e-4, 100, 0)
    f = wl["field"]
    ctx.set_field(f["kind"], f["dir"], f["amp"], f["omega"], f["rate"])
    state = torch.from_numpy(h).cuda()
    out = torch.empty_like(state)
    iters = []
    for _ in range(warmup):
        st, it = ctx.rhs(state, t, out)
        assert st == 0, ctx.last_error()
    torch.cuda.synchronize()
    ctx.prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st, it = ctx.rhs(state, t, out)
        assert st == 0, ctx.last_error()
        iters.append(it)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.prof_read()
    ctx.prof_enable(False)
    res = dict(value=steps / dt, ms_per_step=1e3 * dt / steps, inner_iters=float(np.mean(iters)), prof=prof)
    del out, state
    ctx.close()
    return res


def cpu_baseline(wl, mat, jc, h, t, iters):
    """The oracle as it stands, one core: time its stencil (Faraday + power law)
    and one inner iteration of (18) at the full workload size, scaled to one
    right-hand side with the GPU's mean iteration count."""
    from oracle import bulk
    from oracle.field import AppliedField
    f = wl["field"]
    nx, ny, nz = wl["n"]
    prob = bulk.BulkProblem(nx, ny, nz, *wl["L"], mat, jc_cell=jc, n=wl["nexp"], rho_out=1.0, tol=1e-4,
                            fixed_iters=1, field=AppliedField(f["kind"], f["dir"], f["amp"], f["omega"], f["rate"]))
    t0 = time.perf_counter()
    bulk.hdot_in(prob, h)
    t_st = time.perf_counter() - t0
    t0 = time.perf_counter()
    bulk.rhs(prob, h, t)
    t_one = time.perf_counter() - t0
    t_it = max(t_one - t_st, 1e-9)
    per_rhs = t_st + iters * t_it
    return dict(value=1.0 / per_rhs, unit="RHS evals/s", cores=1, kind="oracle",
                sample="one stencil pass (%.1f s) and one inner iteration (%.1f s) of the NumPy FP64 oracle at "
                       "256^3, scaled to %.2f iterations per RHS" % (t_st, t_it, iters))


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the method is benchmarked on a single MI355X "
              "(multi-GPU sharding is a design note, not a measured path).", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available()
    wl, mat, jc, h = bulk_inputs(a.workload, a.t)
    lo, hi = box_of(mat)
    geo = dict(n=wl["n"], box0=lo, box1=hi)
    res = {}
    for prec in (["mixed"] if a.no_fp64 else ["mixed", "fp64"]):
        res[prec] = run_gpu(prec, wl, mat, jc, h, a.steps, a.warmup, a.t)
        print("[bench] %s: %.1f RHS/s, %.3f ms/RHS, %.2f inner iterations" %
              (prec, res[prec]["value"], res[prec]["ms_per_step"], res[prec]["inner_iters"]), file=sys.stderr,
              flush=True)
    m = res["mixed"]
    # dominant kernel by total recorded time
    kern = max((k for k in m["prof"] if alg_bytes(k, geo, "mixed")), key=lambda k: m["prof"][k][1])
    cnt, tot = m["prof"][kern]
    avg_s = tot / cnt * 1e-3
    ab = alg_bytes(kern, geo, "mixed")
    achieved = ab / avg_s / 1e9
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None, kernel=kern,
                bytes_per_launch=ab, avg_launch_us=round(avg_s * 1e6, 2))
    per_kernel = {k: dict(launches=v[0], avg_us=round(v[1] / v[0] * 1e3, 2),
                          GBps=(round(alg_bytes(k, geo, "mixed") / (v[1] / v[0] * 1e-3) / 1e9, 1)
                                if alg_bytes(k, geo, "mixed") else None)) for k, v in m["prof"].items()}
    line = dict(metric="RHS evals/s at 256^3 padded grid (mixed vs FP64) + adjoint/forward time ratio",
                value=round(m["value"], 3), unit="RHS evals/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
                ms_per_step=round(m["ms_per_step"], 4), higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f32+f64", data="synthetic",
                config=dict(workload="%s: 128^3-cell cube in a 256^3 periodic grid, n=50, ramp tilted 30 deg, "
                                     "log-normal jc (s=0.15, l=6 cells), Bean-like snapshot at t=%g" % (a.workload, a.t),
                            precision="mixed", inner_tol=1e-4),
                inner_iters=round(m["inner_iters"], 3),
                roofline=roof, kernels_mixed=per_kernel)
    if "fp64" in res:
        line["fp64"] = dict(value=round(res["fp64"]["value"], 3), ms_per_step=round(res["fp64"]["ms_per_step"], 4),
                            inner_iters=round(res["fp64"]["inner_iters"], 3))
        line["mixed_over_fp64"] = round(m["value"] / res["fp64"]["value"], 3)
    line["adjoint_forward_ratio"] = None
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(wl, mat, jc, h, a.t, m["inner_iters"])
    line["host"] = dict(cpu=platform.processor() or platform.machine(), cpu_count=os.cpu_count(),
                        numpy=np.__version__)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
