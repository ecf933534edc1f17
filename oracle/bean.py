"""Bean critical-state closed forms for thin films.  TEST INFRASTRUCTURE ONLY.

The power law (3) tends to the Bean model as n -> infinity (Sec. 2.3); the
paper validates its film solver against the analytic Bean solutions for a thin
disk [refs 23, 24] and an infinite strip [ref 27] after a monotone field rise
from the virgin state.  Dimensionless sheet critical current jc, applied
field ha (both in units of jc, Sec. 2.3).  Signs: the field rises along +z,
so the screening current circulates clockwise seen from +z.

Strip of half-width w, infinite along x (coordinate y across it):
  flux front  b = w / cosh(pi ha / jc)
  j_x(y) = (2 jc / pi) arctan( y sqrt(w^2 - b^2) / (w sqrt(b^2 - y^2)) ),  |y| < b
  j_x(y) = jc sign(y),                                                     b <= |y| <= w
  h_z(y) = 0                                                               |y| < b
  h_z(y) = (jc/pi) artanh( w sqrt(y^2 - b^2) / (|y| sqrt(w^2 - b^2)) )     b < |y| < w
  h_z(y) = (jc/pi) artanh( |y| sqrt(w^2 - b^2) / (w sqrt(y^2 - b^2)) )     |y| > w

Disk of radius R (azimuthal current, positive = counter-clockwise):
  flux front  a = R / cosh(2 ha / jc)
  j_phi(r) = -(2 jc / pi) arctan( (r / R) sqrt((R^2 - a^2) / (a^2 - r^2)) ),  r < a
  j_phi(r) = -jc,                                                             a <= r <= R
  h_z(r) in the film plane: ha plus the field of that current, the disk taken
  as coaxial current loops (Biot-Savart law): a loop of radius s carrying a
  unit current gives, at radius r in its plane,
    (1 / 2 pi) [ K(m) / (s + r) + E(m) / (s - r) ],  m = 4 s r / (s + r)^2,
  with K, E the complete elliptic integrals (parameter m); the E term is a
  principal value at s = r.
"""
import numpy as np
from scipy import integrate, special


def strip_front(w, ha, jc=1.0):
    return w / np.cosh(np.pi * ha / jc)


def strip_current(y, w, ha, jc=1.0):
    y = np.asarray(y, dtype=np.float64)
    b = strip_front(w, ha, jc)
    out = np.zeros_like(y)
    ay = np.abs(y)
    inner = ay < b
    yi = y[inner]
    out[inner] = (2 * jc / np.pi) * np.arctan(yi * np.sqrt(w * w - b * b) / (w * np.sqrt(b * b - yi * yi)))
    band = (ay >= b) & (ay <= w)
    out[band] = jc * np.sign(y[band])
    return out


def strip_field(y, w, ha, jc=1.0):
    y = np.asarray(y, dtype=np.float64)
    b = strip_front(w, ha, jc)
    ay = np.abs(y)
    out = np.zeros_like(y)
    band = (ay > b) & (ay < w)
    yb = ay[band]
    out[band] = (jc / np.pi) * np.arctanh(w * np.sqrt(yb * yb - b * b) / (yb * np.sqrt(w * w - b * b)))
    outside = ay > w
    yo = ay[outside]
    out[outside] = (jc / np.pi) * np.arctanh(yo * np.sqrt(w * w - b * b) / (w * np.sqrt(yo * yo - b * b)))
    return out


def disk_front(R, ha, jc=1.0):
    return R / np.cosh(2.0 * ha / jc)


def disk_current(r, R, ha, jc=1.0):
    r = np.asarray(r, dtype=np.float64)
    a = disk_front(R, ha, jc)
    out = np.zeros_like(r)
    inner = r < a
    ri = r[inner]
    out[inner] = -(2 * jc / np.pi) * np.arctan((ri / R) * np.sqrt((R * R - a * a) / (a * a - ri * ri)))
    band = (r >= a) & (r <= R)
    out[band] = -jc
    return out


def _loop_field_parts(s, r):
    """K / (s + r) and E of the loop kernel above (E still to be divided by s - r)."""
    m = np.minimum(4 * s * r / (s + r) ** 2, 1 - 1e-16)
    return special.ellipk(m) / (s + r), special.ellipe(m)


def disk_field(r, R, ha, jc=1.0, tol=1e-12):
    """h_z(r) of the Bean disk in the film plane (r >= 0, array): the applied
    field plus the field of disk_current by superposition of coaxial loops;
    zero inside the flux front, logarithmically singular at r = R.  tol: the
    quadratures' relative tolerance."""
    a = disk_front(R, ha, jc)
    J = lambda s: float(disk_current(np.array([s]), R, ha, jc)[0])
    out = np.empty(np.shape(r))
    for idx, r0 in np.ndenumerate(np.asarray(r, dtype=np.float64)):
        k_part, lo = 0.0, 0.0
        for hi in sorted({min(r0, R), a, R}):
            if hi > lo:
                k_part += integrate.quad(lambda s: J(s) * _loop_field_parts(s, r0)[0], lo, hi, limit=400,
                                         epsabs=0.1 * tol, epsrel=tol)[0]
                lo = hi
        e_part = integrate.quad(lambda s: J(s) * _loop_field_parts(s, r0)[1], 0.0, R, weight="cauchy", wvar=r0,
                                limit=400, epsabs=0.1 * tol, epsrel=tol)[0]
        out[idx] = ha + (k_part + e_part) / (2 * np.pi)
    return out
