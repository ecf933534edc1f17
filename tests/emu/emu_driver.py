"""Run the CPU-emulated HIP library on small cases and compare with the
oracle.  TEST INFRASTRUCTURE ONLY (run in a subprocess with libasan preloaded,
see tests/test_emu_bounds.py)."""
import ctypes
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from tests._cases import bulk_case, film_case, make_oracle, rel_l2  # noqa: E402
from paper_1801_04869_amd import _lib  # noqa: E402


def load(path):
    L = ctypes.CDLL(path)
    for name, (res, args) in _lib.SIGNATURES.items():
        f = getattr(L, name, None)
        if f is None:
            continue
        f.restype = res
        f.argtypes = args
    L.emu_dev_alloc.restype = ctypes.c_void_p
    L.emu_dev_alloc.argtypes = [ctypes.c_size_t]
    L.emu_dev_free.argtypes = [ctypes.c_void_p]
    L.emu_h2d.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
    L.emu_d2h.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
    global _L
    _L = L
    return L


_L = None


class Dev:
    """A buffer in the emulated device address space (like a torch tensor on
    the GPU): the library must never read it from host code."""

    def __init__(self, arr=None, like=None):
        src = np.ascontiguousarray(arr if arr is not None else np.zeros_like(like))
        self.shape, self.dtype, self.nbytes = src.shape, src.dtype, src.nbytes
        self.ptr = _L.emu_dev_alloc(max(self.nbytes, 1))
        if arr is not None:
            _L.emu_h2d(self.ptr, src.ctypes.data, self.nbytes)

    def numpy(self):
        out = np.empty(self.shape, self.dtype)
        _L.emu_d2h(out.ctypes.data, self.ptr, self.nbytes)
        return out

    def __del__(self):
        if _L is not None and self.ptr:
            _L.emu_dev_free(self.ptr)
            self.ptr = None


def P(a):
    if isinstance(a, Dev):
        return ctypes.c_void_p(a.ptr)
    return ctypes.c_void_p(a.ctypes.data)


def setup(L, case, prec, fixed=0, max_inner=100, tol=None, deriv="staggered"):
    h = ctypes.c_void_p()
    assert L.mag_create(ctypes.byref(h), case["dim"], prec, None) == 0
    nx, ny, nz = case["n"]
    assert L.mag_set_grid(h, nx, ny, nz, *case["L"]) == 0, L.mag_last_error(h)
    if deriv == "spectral":
        assert L.mag_set_derivatives(h, 1, -1.0) == 0, L.mag_last_error(h)
    mat = Dev(np.ascontiguousarray(case["mat"], dtype=np.uint8))
    assert L.mag_set_domain(h, P(mat)) == 0, L.mag_last_error(h)
    jc = None if case["jc"] is None else Dev(np.ascontiguousarray(case["jc"]))
    assert L.mag_set_params(h, None if jc is None else P(jc), 1.0, case["nexp"], 1.0, case["rho_out"]) == 0
    if tol is None:
        tol = 2e-4 if case["dim"] == 2 else 1e-4
    assert L.mag_set_solver(h, 0.7, tol, max_inner, fixed) == 0, L.mag_last_error(h)
    f = case["field"]
    d = (ctypes.c_double * 3)(*[float(v) for v in f["dir"]])
    assert L.mag_set_field(h, f["kind"], d, f["amp"], f["omega"], f["rate"]) == 0
    return h, (mat, jc)


def run_rhs(L, h, state, t):
    s = Dev(np.ascontiguousarray(state, dtype=np.float64))
    out = Dev(like=s.numpy())
    it = ctypes.c_int(0)
    rc = L.mag_rhs(h, P(s), t, P(out), ctypes.byref(it))
    return rc, it.value, out.numpy()


def capture_check(L):
    """mag_integrate_captured (step control on the device, attempts replayed
    from a captured graph) against mag_integrate (host-driven) on the same
    film with a fixed inner count: same accepted and rejected attempts and the
    same final state, bit for bit (host and emulated device share one libm);
    a second run from the same start reuses the graph and repeats the result."""
    fails = 0
    for prec, chunk in ((0, 3), (1, 4), (2, 3)):
        case = film_case(32, 16, L=(2.0, 1.0), kind="offrect", jc_s=0.2, n=19.0)
        case["state"] = np.zeros_like(case["state"])
        res = []
        for mode in ("host", "captured", "captured"):
            h, keep = setup(L, case, prec, fixed=2)
            y = Dev(np.zeros_like(case["state"]))
            if mode == "host":
                ns = ctypes.c_int(0)
                rc = L.mag_integrate(h, P(y), 0.0, 0.02, 1e-3, 1e-6, None, 0, ctypes.byref(ns))
                res.append((rc, ns.value, None, y.numpy()))
            else:
                na, nr, tr = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0)
                rc = L.mag_integrate_captured(h, P(y), 0.0, 0.02, 1e-3, 1e-6, chunk, 100000, ctypes.byref(na),
                                              ctypes.byref(nr), ctypes.byref(tr))
                if rc != 0:
                    print("   captured rc=%d %s" % (rc, L.mag_last_error(h)), flush=True)
                res.append((rc, na.value, tr.value, y.numpy()))
            L.mag_destroy(h)
        (r0, n0, _, y0), (r1, n1, t1, y1), (r2, n2, t2, y2) = res
        ok = r0 == r1 == r2 == 0 and n0 == n1 == n2 and t1 == t2 == 0.02 and np.array_equal(y0, y1) \
            and np.array_equal(y1, y2)
        fails += not ok
        print("capture prec=%d chunk=%d host steps=%d captured steps=%d/%d t=%s max|dy|=%.3e %s" %
              (prec, chunk, n0, n1, n2, t1, float(np.abs(y0 - y1).max()), "ok" if ok else "FAIL"), flush=True)
    return fails


def main(path, which):
    from oracle import bulk, film
    L = load(path)
    fails = 0
    cases = []
    if which in ("bulk", "all"):
        cases += [("bulk", bulk_case(16, 16, 16, half=(0.55, 0.55, 0.55)), 0, 1),
                  ("bulk", bulk_case(32, 16, 16, L=(4.0, 2.0, 2.0), half=(1.3, 0.6, 0.6), shift=(1, 0, -2),
                                     jc_s=0.2), 1, 2),
                  ("bulk-wrap", bulk_case(16, 16, 16, half=(0.55, 0.55, 0.55), shift=(8, 0, 0)), 0, 2)]
    if which in ("bulk32", "all"):
        # the first bulk GPU case: 32^3 cube in a 32^3 grid, n = 25, FP64, one
        # inner iteration, with the GPU test's host call sequence
        cases += [("bulk-32", bulk_case(32, 32, 32, n=25.0), 0, 1)]
    if which in ("bulkgpu", "all"):
        # every bulk case of the GPU parity tests (shapes, precisions, counts)
        for prec in (0, 1):
            for fixed in (1, 3):
                cases += [("bulk-32", bulk_case(32, 32, 32, n=25.0), prec, fixed),
                          ("bulk-64x32x16", bulk_case(64, 32, 16, L=(4.0, 2.0, 1.0), half=(1.3, 0.7, 0.45),
                                                      shift=(1, -2, 3), n=25.0), prec, fixed),
                          ("bulk-16x64x32", bulk_case(16, 64, 32, L=(1.0, 4.0, 2.0), half=(0.45, 1.1, 0.7),
                                                      jc_s=0.2, n=50.0), prec, fixed)]
    if which in ("capture", "all"):
        fails += capture_check(L)
    if which in ("film", "all"):
        cases += [("film", film_case(32, 16, L=(2.0, 1.0), kind="offrect", jc_s=0.2), 0, 2),
                  ("film", film_case(16, 32, L=(1.0, 2.0), kind="ring", rho_out=20.0), 1, 1),
                  ("film", film_case(128, 64, L=(2.0, 1.0), kind="offrect", jc_s=0.2), 0, 2),
                  ("film", film_case(64, 32, L=(2.0, 1.0), kind="ring", jc_s=0.2, rho_out=20.0), 1, 3),
                  # mixed iteration with the final evaluation in double
                  ("film", film_case(32, 16, L=(2.0, 1.0), kind="offrect", jc_s=0.2), 2, 2),
                  ("film", film_case(64, 32, L=(2.0, 1.0), kind="ring", jc_s=0.2, rho_out=20.0), 2, 3),
                  ("film", film_case(64, 32, L=(2.0, 1.0), kind="ring", jc_s=0.2, rho_out=20.0), 2, 1),
                  ("film", film_case(32, 16, L=(2.0, 1.0), kind="offrect", jc_s=0.2), 2, 0),
                  # column passes of 1024 and 2048 rows: two column groups per block
                  ("film", film_case(16, 1024, L=(0.25, 2.0), kind="offrect", jc_s=0.2), 1, 2),
                  ("film", film_case(16, 2048, L=(0.25, 2.0), kind="offrect", jc_s=0.2), 0, 1)]
    if which in ("spectral", "all"):
        # the spectral form of Sec. 2.2 (fields on the nodes, filtered Fourier
        # derivatives), every precision, fixed counts and the stop test
        sp = "spectral"
        cases += [("spectral", film_case(32, 16, L=(2.0, 1.0), kind="offrect", jc_s=0.2), 0, 2, sp),
                  ("spectral", film_case(16, 32, L=(1.0, 2.0), kind="ring", rho_out=20.0), 1, 1, sp),
                  ("spectral", film_case(64, 32, L=(2.0, 1.0), kind="ring", jc_s=0.2, rho_out=20.0), 2, 3, sp),
                  ("spectral", film_case(32, 32, L=(1.0, 1.0), kind="disk"), 0, 0, sp),
                  ("spectral", film_case(32, 32, L=(1.0, 1.0), kind="disk"), 2, 0, sp),
                  ("spectral", film_case(16, 1024, L=(0.25, 2.0), kind="offrect", jc_s=0.2), 1, 2, sp)]
    if which in ("radix3", "all"):
        # grids of 3 * 2^k nodes (radix-12 first stage): both aspect ratios,
        # every precision, both film forms, the stop test
        sp = "spectral"
        cases += [("radix3", film_case(96, 64, L=(2.25, 1.5), kind="hole", jc_s=0.2, rho_out=20.0), 0, 2),
                  ("radix3", film_case(64, 96, L=(1.5, 2.25), kind="offrect", jc_s=0.2), 1, 3),
                  ("radix3", film_case(48, 48, L=(1.0, 1.0), kind="disk"), 2, 2),
                  ("radix3", film_case(96, 48, L=(2.0, 1.0), kind="offrect", jc_s=0.2), 0, 0),
                  ("radix3", film_case(96, 64, L=(2.25, 1.5), kind="hole", jc_s=0.2, rho_out=20.0), 1, 2, sp),
                  ("radix3", film_case(48, 96, L=(1.0, 2.0), kind="ring", rho_out=20.0), 0, 0, sp)]
    for entry in cases:
        name, case, prec, fixed = entry[:4]
        deriv = entry[4] if len(entry) > 4 else "staggered"
        h, keep = setup(L, case, prec, fixed=fixed, deriv=deriv)
        rc, it, out = run_rhs(L, h, case["state"], 0.2)
        prob = make_oracle(case, fixed=fixed, deriv=deriv)
        mod = film if case["dim"] == 2 else bulk
        ref, rit, rst = mod.rhs(prob, case["state"], 0.2)
        err = rel_l2(out, ref)
        tol = 1e-10 if prec == 0 else 1e-4
        if fixed == 0 and it != rit:
            tol = 10 * 2e-4   # a mixed form may stop one evaluation apart from the oracle
        ok = rc == 0 and (it == fixed if fixed else it >= 1) and err < tol
        fails += not ok
        print("%-10s n=%s prec=%d fixed=%d rc=%d it=%d rel-L2=%.3e %s" % (name, case["n"], prec, fixed, rc, it, err,
                                                                         "ok" if ok else "FAIL"), flush=True)
        if case["dim"] == 2:
            # vector-Jacobian product against the oracle's transpose
            from oracle import adjoint
            ybar_h = np.random.default_rng(7).standard_normal(case["state"].shape)
            ybar = Dev(ybar_h)
            gb_d = Dev(like=ybar_h)
            jb_d = Dev(like=ybar_h)
            s_ = Dev(np.ascontiguousarray(case["state"]))
            rc = L.mag_rhs_vjp(h, P(s_), 0.2, P(ybar), P(gb_d), P(jb_d))
            gb, jb = gb_d.numpy(), jb_d.numpy()
            ybar = ybar_h
            rg, rj, rcnt, rst = adjoint.film_rhs_vjp(prob, case["state"], 0.2, ybar)
            e1 = rel_l2(gb, rg)
            e2 = rel_l2(jb, rj) if case["jc"] is not None else 0.0
            okv = rc == 0 and e1 < tol and e2 < tol
            fails += not okv
            print("   vjp rc=%d rel-L2 g=%.3e jc=%.3e %s" % (rc, e1, e2, "ok" if okv else "FAIL"), flush=True)
        # observables
        m = (ctypes.c_double * 3)()
        s = Dev(np.ascontiguousarray(case["state"]))
        nn = int(np.prod(case["n"]))
        hz = Dev(np.zeros(nn))
        jj = Dev(np.zeros(case["dim"] * nn))
        rc = L.mag_observe(h, P(s), 0.3, P(hz), P(jj), m)
        print("   observe rc=%d m=%s" % (rc, list(m)), flush=True)
        if case["dim"] == 2:
            rhz, (rjx, rjy), rmz = film.observe(prob, case["state"], 0.3)
            eo = max(rel_l2(hz.numpy(), rhz.ravel()), rel_l2(jj.numpy(), np.concatenate([rjx.ravel(), rjy.ravel()])))
            oko = rc == 0 and eo < (1e-10 if prec == 0 else 1e-5)
            fails += not oko
            print("   observe vs oracle rel-L2=%.3e %s" % (eo, "ok" if oko else "FAIL"), flush=True)
        if case["dim"] == 2:
            # the allocation-free moment against mag_observe's
            md = Dev(np.full(3, np.nan))
            nx, ny, _ = case["n"]
            rc2 = L.mag_film_moment_noalloc(P(s), nx, ny, case["L"][0], case["L"][1], P(md), None)
            mn = md.numpy()
            okm = rc2 == 0 and mn[0] == 0 and mn[1] == 0 and abs(mn[2] - m[2]) <= 1e-13 * max(abs(m[2]), 1e-300)
            fails += not okm
            print("   noalloc moment rc=%d m=%s %s" % (rc2, list(mn), "ok" if okm else "FAIL"), flush=True)
        L.mag_destroy(h)
    print("EMU_DONE fails=%d" % fails, flush=True)
    return fails


if __name__ == "__main__":
    sys.exit(1 if main(sys.argv[1], sys.argv[2] if len(sys.argv) > 2 else "all") else 0)
