"""Thin Python binding of the magfft C ABI (include/magfft.h).

PyTorch provides device memory and the HIP stream only; every step of the
right-hand side, the time stepping and the observables runs in the HIP
library.  Names mirror the C functions.
"""
import ctypes

import torch

from . import _lib

OK, NOT_CONVERGED, STEP_UNDERFLOW = 0, 1, 2
E_ARG, E_STATE, E_HIP, E_NOMEM, E_NUMERIC = -1, -2, -3, -4, -5
FP64, MIXED, MIXED_FINAL64 = 0, 1, 2
RAMP, SINE, ROTATE = 0, 1, 2
STAGGERED, SPECTRAL = 0, 1


class MagError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("magfft error %d: %s" % (code, msg))
        self.code = code


def _ptr(t, dtype):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.device.type != "cuda":
        raise ValueError("expected a contiguous %s tensor on the GPU" % dtype)
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One problem: a film (dim 2) or a bulk sample (dim 3) on one GPU."""

    def __init__(self, dim, precision=FP64, stream=None):
        self._L = _lib.lib()
        self._h = ctypes.c_void_p()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        rc = self._L.mag_create(ctypes.byref(self._h), int(dim), int(precision), ctypes.c_void_p(stream.cuda_stream))
        if rc != OK:
            raise MagError(rc, "mag_create failed")
        self.dim = dim
        self.precision = precision
        self.shape = None

    def close(self):
        if self._h:
            self._L.mag_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=(OK,)):
        if rc in allow:
            return rc
        raise MagError(rc, self._L.mag_last_error(self._h).decode())

    def last_error(self):
        return self._L.mag_last_error(self._h).decode()

    # ---------------------------------------------------------- setup
    def set_grid(self, nx, ny, nz, Lx, Ly, Lz=1.0):
        self._check(self._L.mag_set_grid(self._h, nx, ny, nz, Lx, Ly, Lz))
        self.n = (nx, ny, nz)
        self.shape = (ny, nx) if self.dim == 2 else (3, nz, ny, nx)

    def set_domain(self, material):
        self._check(self._L.mag_set_domain(self._h, _ptr(material, torch.uint8)))

    def set_params(self, jc_map=None, jc0=1.0, n=19.0, e0=1.0, rho_out=1.0):
        self._check(self._L.mag_set_params(self._h, _ptr(jc_map, torch.float64), jc0, n, e0, rho_out))
        self.params = (jc_map, jc0, n, e0, rho_out)

    def set_solver(self, lam=0.7, tol=None, max_inner=100, fixed_iters=0):
        if tol is None:
            tol = 2e-4 if self.dim == 2 else 1e-4
        self._check(self._L.mag_set_solver(self._h, lam, tol, max_inner, fixed_iters))

    def set_field(self, kind=RAMP, direction=(0.0, 0.0, 1.0), amp=1.0, omega=1.0, rate=1.0):
        d = (ctypes.c_double * 3)(*[float(v) for v in direction])
        self._check(self._L.mag_set_field(self._h, kind, d, amp, omega, rate))

    # ---------------------------------------------------------- evaluation
    def rhs(self, state, t, out, wait=True):
        """out = f(state, t); returns (status, n_inner); status OK or NOT_CONVERGED.
        wait=False with a fixed iteration count: enqueue only (n_inner None);
        rhs_status() reports the outcome."""
        it = ctypes.c_int(0)
        rc = self._L.mag_rhs(self._h, _ptr(state, torch.float64), float(t), _ptr(out, torch.float64),
                             ctypes.byref(it) if wait else None)
        self._check(rc, allow=(OK, NOT_CONVERGED))
        return rc, (it.value if wait else None)

    def rhs_status(self):
        it = ctypes.c_int(0)
        rc = self._L.mag_rhs_status(self._h, ctypes.byref(it))
        self._check(rc)
        return rc, it.value

    def step(self, state, t, dt, rtol=1e-3, atol=1e-6):
        """One step attempt; returns (t, dt_next, accepted)."""
        tt, dd, acc = ctypes.c_double(t), ctypes.c_double(dt), ctypes.c_int(0)
        rc = self._L.mag_step(self._h, _ptr(state, torch.float64), ctypes.byref(tt), ctypes.byref(dd),
                              rtol, atol, ctypes.byref(acc))
        self._check(rc)
        return tt.value, dd.value, bool(acc.value)

    def integrate(self, state, t0, t1, rtol=1e-3, atol=1e-6, obs_cap=0):
        """Integrate in place; returns (n_steps, obs) with obs rows (t, dt, mx, my, mz, n_inner)."""
        ns = ctypes.c_int(0)
        obs = (ctypes.c_double * (6 * obs_cap))() if obs_cap > 0 else None
        rc = self._L.mag_integrate(self._h, _ptr(state, torch.float64), t0, t1, rtol, atol,
                                   ctypes.cast(obs, _lib.P_double) if obs is not None else None, obs_cap,
                                   ctypes.byref(ns))
        self._check(rc)
        rows = []
        if obs is not None:
            for i in range(min(ns.value, obs_cap)):
                rows.append(tuple(obs[6 * i:6 * i + 6]))
        return ns.value, rows

    def integrate_captured(self, state, t0, t1, rtol=1e-3, atol=1e-6, chunk=16, max_attempts=10 ** 7):
        """Integrate in place with the step control on the device, step
        attempts replayed from a captured graph (film, fixed inner count);
        returns (accepted, rejected, t reached); t reached < t1 when
        max_attempts ran out first."""
        na, nr, tr = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0)
        rc = self._L.mag_integrate_captured(self._h, _ptr(state, torch.float64), float(t0), float(t1), rtol, atol,
                                            int(chunk), int(max_attempts), ctypes.byref(na), ctypes.byref(nr),
                                            ctypes.byref(tr))
        # NOT_CONVERGED here means max_attempts ran out before t1
        self._check(rc, allow=(OK, NOT_CONVERGED))
        return na.value, nr.value, tr.value

    def observe(self, state, t, want_hz=True, want_j=True):
        """Returns (hz, j, m): hz on nodes (2D) / z-edges (3D), j on edges/faces
        (2 or 3 component planes), m the magnetic moment (host tuple)."""
        dev = state.device
        nx, ny, nz = self.n
        grid = (ny, nx) if self.dim == 2 else (nz, ny, nx)
        hz = torch.empty(grid, dtype=torch.float64, device=dev) if want_hz else None
        j = torch.empty((self.dim,) + grid, dtype=torch.float64, device=dev) if want_j else None
        m = (ctypes.c_double * 3)()
        self._check(self._L.mag_observe(self._h, _ptr(state, torch.float64), float(t), _ptr(hz, torch.float64),
                                        _ptr(j, torch.float64), m))
        return hz, j, (m[0], m[1], m[2])

    def rhs_vjp(self, state, t, out_bar, state_bar, jc_bar=None):
        rc = self._L.mag_rhs_vjp(self._h, _ptr(state, torch.float64), float(t), _ptr(out_bar, torch.float64),
                                 _ptr(state_bar, torch.float64), _ptr(jc_bar, torch.float64))
        self._check(rc, allow=(OK, NOT_CONVERGED))
        return rc

    def reset_warm_start(self):
        self._check(self._L.mag_reset_warm_start(self._h))

    def set_warm_start(self, on=True):
        self._check(self._L.mag_set_warm_start(self._h, 1 if on else 0))

    def set_derivatives(self, mode, sigma=-1.0):
        """Film discretisation: STAGGERED differences or the SPECTRAL form of
        Sec. 2.2 (sigma < 0: the width sqrt(dx^2 + dy^2))."""
        self._check(self._L.mag_set_derivatives(self._h, int(mode), float(sigma)))

    def step_fixed(self, state, t, dt):
        """One step of exactly dt without error control (state advances in place)."""
        return self._check(self._L.mag_step_fixed(self._h, _ptr(state, torch.float64), float(t), float(dt)),
                           allow=(OK, NOT_CONVERGED))

    def step_vjp(self, state, t, dt, ybar_new, ybar, jc_bar=None):
        """ybar = (d step / d state)^T ybar_new; jc_bar += jc-map cotangent."""
        return self._check(self._L.mag_step_vjp(self._h, _ptr(state, torch.float64), float(t), float(dt),
                                                _ptr(ybar_new, torch.float64), _ptr(ybar, torch.float64),
                                                _ptr(jc_bar, torch.float64)), allow=(OK, NOT_CONVERGED))

    def observe_vjp(self, hz_bar, state_bar):
        self._check(self._L.mag_observe_vjp(self._h, _ptr(hz_bar, torch.float64), _ptr(state_bar, torch.float64)))

    # ---------------------------------------------------------- instrumentation
    def stats(self, reset=False):
        """(right-hand sides, inner iterations) evaluated since the last reset."""
        a, b = ctypes.c_longlong(0), ctypes.c_longlong(0)
        self._check(self._L.mag_stats(self._h, 1 if reset else 0, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def prof_enable(self, on=True, only=None):
        """Record HIP events around kernel launches: all kernels, or only the
        kernel named `only`."""
        mode = 0
        if on:
            mode = 1 if only is None else 2 + self.kernel_id(only)
        self._check(self._L.mag_prof_enable(self._h, mode))

    def kernel_id(self, name):
        k = 0
        while True:
            n = self._L.mag_prof_kernel_name(k)
            if n is None:
                raise KeyError(name)
            if n.decode() == name:
                return k
            k += 1

    def prof_read(self):
        """{kernel name: (launches, total ms)} for kernels with recorded launches."""
        out = {}
        k = 0
        while True:
            name = self._L.mag_prof_kernel_name(k)
            if name is None:
                break
            cnt, ms = ctypes.c_int(0), ctypes.c_double(0)
            self._check(self._L.mag_prof_read(self._h, k, ctypes.byref(cnt), ctypes.byref(ms)))
            if cnt.value:
                out[name.decode()] = (cnt.value, ms.value)
            k += 1
        return out
