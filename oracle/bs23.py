"""Explicit Runge-Kutta 3(2) pair of Bogacki and Shampine with step control.
TEST INFRASTRUCTURE ONLY.

The paper integrates the method-of-lines system with Matlab's ode23 at its
default tolerances, rtol 1e-3 and atol 1e-6 (Sec. 2.2 and 3.1).  ode23 is the
Bogacki-Shampine 3(2) pair (Bogacki & Shampine, Appl. Math. Lett. 2 (1989)
321-325) with the first-same-as-last property.  The controller constants are
not given in the paper; this module fixes its own (stated below) and the GPU
driver uses the same ones:

* error norm  max_i |err_i| / max(rtol * max(|y_i|, |ynew_i|), atol); accept if <= 1;
  a non-finite norm (overflow in a stage) counts as infinite
* accepted:   h <- h * min(5, max(0.2, 0.8 * err^(-1/3)))   (factor 5 when err = 0)
* rejected:   h <- h * max(0.2, 0.8 * err^(-1/3))
* right-hand side not converged (status != 0): reject, h <- h / 2
* the last step is stretched to land on t1 when 1.1 h >= t1 - t
* first step: min(0.1 (t1 - t0), 0.8 rtol^(1/3) / max_i(|f_i| / max(|y_i|, atol/rtol)))
"""
import numpy as np

# Butcher tableau of the 3(2) pair
C2, C3 = 0.5, 0.75
A21, A32 = 0.5, 0.75
B1, B2, B3 = 2.0 / 9.0, 1.0 / 3.0, 4.0 / 9.0
E1, E2, E3, E4 = -5.0 / 72.0, 1.0 / 12.0, 1.0 / 9.0, -1.0 / 8.0

ACCEPTED, REJECTED, RHS_FAILED = 0, 1, 2


def error_norm(err, y, ynew, rtol, atol):
    scale = np.maximum(rtol * np.maximum(np.abs(y), np.abs(ynew)), atol)
    en = float(np.max(np.abs(err) / scale))
    return en if np.isfinite(en) else np.inf         # overflow in a stage counts as a failed step


def attempt(f, t, y, h, k1):
    """One step attempt from (t, y) with step h and k1 = f(t, y).

    ``f(t, y)`` returns (value, status).  Returns (ynew, k4, err, status)."""
    k2, st = f(t + C2 * h, y + (A21 * h) * k1)
    if st != 0:
        return None, None, None, RHS_FAILED
    k3, st = f(t + C3 * h, y + (A32 * h) * k2)
    if st != 0:
        return None, None, None, RHS_FAILED
    ynew = y + h * (B1 * k1 + B2 * k2 + B3 * k3)
    k4, st = f(t + h, ynew)
    if st != 0:
        return None, None, None, RHS_FAILED
    err = h * (E1 * k1 + E2 * k2 + E3 * k3 + E4 * k4)
    return ynew, k4, err, 0


def new_step(h, en, accepted):
    if accepted:
        fac = 5.0 if en == 0.0 else min(5.0, max(0.2, 0.8 * en ** (-1.0 / 3.0)))
    else:
        fac = max(0.2, 0.8 * en ** (-1.0 / 3.0))
    return h * fac


def first_step(t0, t1, y0, f0, rtol, atol):
    span = abs(t1 - t0)
    rh = float(np.max(np.abs(f0) / np.maximum(np.abs(y0), atol / rtol))) / (0.8 * rtol ** (1.0 / 3.0))
    h = 0.1 * span
    if rh * h > 1.0:
        h = 1.0 / rh
    return h


def integrate(f, y0, t0, t1, rtol=1e-3, atol=1e-6, h0=None, replay=None, max_steps=10 ** 7,
              on_step=None):
    """Integrate y' = f(t, y) from t0 to t1.

    ``replay``: optional sequence of step sizes taken as accepted without
    error control (used to compare two implementations on one time grid).
    ``on_step(t, y, h)`` is called after each accepted step.
    Returns (y, t, history) with history a list of (t, h, err_norm).
    """
    y = np.array(y0, dtype=np.float64)
    t = float(t0)
    k1, st = f(t, y)
    if st != 0:
        raise RuntimeError("right-hand side failed at the initial point")
    hist = []
    if replay is not None:
        for h in replay:
            ynew, k4, err, st = attempt(f, t, y, h, k1)
            if st != 0:
                raise RuntimeError("right-hand side failed in replay")
            en = error_norm(err, y, ynew, rtol, atol)
            t = t + h
            y, k1 = ynew, k4
            hist.append((t, h, en))
            if on_step is not None:
                on_step(t, y, h)
        return y, t, hist
    h = first_step(t0, t1, y, k1, rtol, atol) if h0 is None else float(h0)
    steps = 0
    while t < t1 and steps < max_steps:
        if 1.1 * h >= t1 - t:
            h = t1 - t
        if h <= 16 * np.finfo(float).eps * max(abs(t), 1.0):
            raise RuntimeError("step size underflow")
        ynew, k4, err, st = attempt(f, t, y, h, k1)
        steps += 1
        if st != 0:
            h = 0.5 * h
            continue
        en = error_norm(err, y, ynew, rtol, atol)
        if en <= 1.0:
            t = t + h
            y, k1 = ynew, k4
            hist.append((t, h, en))
            if on_step is not None:
                on_step(t, y, h)
            h = new_step(h, en, True)
        else:
            h = new_step(h, en, False)
    return y, t, hist
