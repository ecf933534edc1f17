"""Pins of oracle parts that the other CPU tests leave open: the film and bulk
magnetic moments, the transpose of the film h_z map, and the Bean thin-disk
and strip closed forms.  Each pin uses a fact that does not come from the
formula under test (summation by parts on the staggered lattice, the moment
of a current loop, the symmetry of an operator checked through the forward
map that the library mirrors, the flux-free core of the critical state
checked by direct Biot-Savart integration)."""
import numpy as np
import pytest
from scipy import integrate, special

from oracle import adjoint, bean, bulk, film
from paper_1801_04869_amd import workloads as W


def _film(nx=48, ny=40, Lx=1.5, Ly=1.25):
    m = W.film_rect(nx, ny, Lx, Ly, 0.6 * Lx, 0.5 * Ly)
    return film.FilmProblem(nx, ny, Lx, Ly, m)


def _compact(shape, margin, seed):
    """Random field that vanishes within `margin` nodes of the box faces."""
    a = np.random.default_rng(seed).standard_normal(shape)
    sl = tuple(slice(margin, s - margin) for s in shape)
    out = np.zeros(shape)
    out[sl] = a[sl]
    return out


# ------------------------------------------------------------ film moment
def test_film_moment_is_half_r_cross_j_on_the_edges():
    """m_z = (1/2) sum (x j_y - y j_x) dx dy over the staggered edges, with each
    current component taken at its own edge midpoint (Sec. 2.1, eq. (2)).
    Summation by parts makes this equal to sum g dx dy for any g that
    vanishes near the box boundary."""
    p = _film()
    g = _compact((p.ny, p.nx), 2, 3)
    _, (jx, jy), mz = film.observe(p, g, 0.0)
    xn = -p.Lx + p.dx * np.arange(p.nx)
    yn = -p.Ly + p.dy * np.arange(p.ny)
    # j_x at (x_p, y_{q+1/2}); j_y at (x_{p+1/2}, y_q)
    y_xe = (yn + 0.5 * p.dy)[:, None] + 0 * xn[None, :]
    x_ye = (xn + 0.5 * p.dx)[None, :] + 0 * yn[:, None]
    ref = 0.5 * (np.sum(x_ye * jy) - np.sum(y_xe * jx)) * p.dx * p.dy
    assert abs(mz - ref) < 1e-12 * np.abs(g).sum() * p.dx * p.dy


@pytest.mark.parametrize("I", [1.0, -0.37])
def test_film_moment_of_a_uniform_patch_is_current_times_area(I):
    """g = I on a rectangle of nodes and 0 elsewhere is a single loop of
    current I running along the edge midpoints around the rectangle; its
    moment is I times the enclosed area (number of nodes times dx dy)."""
    p = _film()
    g = np.zeros((p.ny, p.nx))
    q0, q1, p0, p1 = 9, 27, 7, 31
    g[q0:q1 + 1, p0:p1 + 1] = I
    _, (jx, jy), mz = film.observe(p, g, 0.0)
    area = (p1 - p0 + 1) * p.dx * (q1 - q0 + 1) * p.dy
    assert abs(mz - I * area) < 1e-13 * area
    # the loop carries current I: |j| dy summed across one side equals |I|
    assert abs(np.abs(jy[(q0 + q1) // 2, :]).sum() * p.dx - 2 * abs(I)) < 1e-12


# ------------------------------------------------------------ bulk moment
def _bulk(n=(20, 16, 12), L=(1.25, 1.0, 0.75)):
    nx, ny, nz = n
    m = W.bulk_box(nx, ny, nz, *L, 0.5 * L[0], 0.5 * L[1], 0.5 * L[2])
    return bulk.BulkProblem(nx, ny, nz, *L, m)


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_bulk_moment_of_a_curl_is_the_integral_of_its_potential(comp):
    """j = C(psi e_c) is the current of the magnetisation psi e_c, whose moment
    is (integral of psi dV) e_c; on the lattice this holds exactly by
    summation by parts for psi supported away from the box faces."""
    p = _bulk()
    psi = _compact(p.shape, 2, 11 + comp)
    h = np.zeros((3,) + p.shape)
    h[comp] = psi
    _, j, m = bulk.observe(p, h, 0.0)
    dV = p.dx * p.dy * p.dz
    ref = np.zeros(3)
    ref[comp] = psi.sum() * dV
    assert np.abs(m - ref).max() < 1e-12 * np.abs(psi).sum() * dV


def test_bulk_moment_of_a_current_loop():
    """A uniform h_z patch on a box of z-edges is a stack of square loops; one
    layer of thickness dz carrying I dz has moment I dz times the enclosed
    area."""
    p = _bulk()
    h = np.zeros((3,) + p.shape)
    I = 0.8
    r0, q0, q1, p0, p1 = 5, 4, 10, 6, 13
    h[2, r0, q0:q1 + 1, p0:p1 + 1] = I
    _, j, m = bulk.observe(p, h, 0.0)
    area = (p1 - p0 + 1) * p.dx * (q1 - q0 + 1) * p.dy
    assert abs(m[2] - I * area * p.dz) < 1e-13 * area
    assert abs(m[0]) < 1e-13 and abs(m[1]) < 1e-13


# ------------------------------------------------------------ h_z transpose
def test_film_hz_vjp_is_the_transpose_of_observe():
    """<hz_bar, dh_z(g)> = <film_hz_vjp(hz_bar), g> with h_z from observe()
    (the forward map h_z = h_e + F^-1[|k|/2 F g] of Sec. 2.1)."""
    p = _film()
    rng = np.random.default_rng(5)
    g = rng.standard_normal((p.ny, p.nx))
    a = rng.standard_normal((p.ny, p.nx))
    he = float(p.field.h(0.3)[2])
    hz, _, _ = film.observe(p, g, 0.3)
    lhs = np.sum(a * (hz - he))
    rhs = np.sum(adjoint.film_hz_vjp(p, a) * g)
    assert abs(lhs - rhs) < 1e-12 * np.sqrt(np.sum(a * a) * np.sum(hz * hz))


def test_film_hz_vjp_rejects_the_other_multiplier():
    """The pin above separates |k|/2 from 2/|k|: the two transposes differ."""
    p = _film()
    a = np.random.default_rng(6).standard_normal((p.ny, p.nx))
    wrong = film.apply_multiplier(a, p.K1)
    assert np.linalg.norm(wrong - adjoint.film_hz_vjp(p, a)) > 0.1 * np.linalg.norm(wrong)


# ------------------------------------------------------------ Bean closed forms
def _ring_hz(rho, r):
    """h_z in the plane at radius r of a unit ring current of radius rho, split
    as K-part (log-singular) and E-part (to be divided by rho - r)."""
    m = 4 * rho * r / (rho + r) ** 2
    m = np.minimum(m, 1 - 1e-16)
    return special.ellipk(m) / (rho + r), special.ellipe(m)


def _disk_hz(r0, R, ha):
    return float(bean.disk_field(np.array([r0]), R, ha)[0])


@pytest.mark.parametrize("ha", [0.3, 0.6])
def test_bean_disk_has_a_flux_free_core(ha):
    """Critical state of a thin disk after a field rise from the virgin state
    (the n -> infinity limit of Sec. 2.3): the disk current must cancel the
    applied field everywhere inside the flux front a, and not outside it."""
    R = 1.0
    a = bean.disk_front(R, ha)
    for r0 in (0.1 * a, 0.5 * a, 0.8 * a):
        assert abs(_disk_hz(r0, R, ha)) < 2e-6 * ha
    # beyond the front the field has penetrated
    assert _disk_hz(0.5 * (a + R), R, ha) > 0.05 * ha


def test_bean_disk_wrong_front_is_rejected():
    """The same check fails for a front shifted by the strip's pi/2 factor."""
    R, ha = 1.0, 0.3
    a_wrong = R / np.cosh(np.pi * ha)
    a = bean.disk_front(R, ha)
    J = lambda rho: -(2 / np.pi) * np.arctan((rho / R) * np.sqrt((R * R - a_wrong ** 2) / (a_wrong ** 2 - rho ** 2))) \
        if rho < a_wrong else (-1.0 if rho <= R else 0.0)
    r0 = 0.5 * min(a, a_wrong)
    k_part = integrate.quad(lambda s: J(s) * _ring_hz(s, r0)[0], 0, R, points=[r0, a_wrong], limit=400)[0]
    e_part = integrate.quad(lambda s: J(s) * _ring_hz(s, r0)[1], 0, R, weight="cauchy", wvar=r0, limit=400)[0]
    assert abs(ha + (k_part + e_part) / (2 * np.pi)) > 1e-3


@pytest.mark.parametrize("ha", [0.2, 0.5])
def test_bean_strip_field_and_flux_free_core(ha):
    """Infinite strip: the field of the Bean current (line-current kernel
    1 / (2 pi (y0 - y))) plus the applied field vanishes for |y0| < b and
    equals strip_field() outside the front."""
    w = 1.0
    b = bean.strip_front(w, ha)
    J = lambda y: float(bean.strip_current(np.array([y]), w, ha)[0])

    def hz(y0):
        pv = integrate.quad(J, -w, w, weight="cauchy", wvar=y0, limit=400, epsabs=1e-13, epsrel=1e-12)[0]
        return ha - pv / (2 * np.pi)

    for y0 in (0.0, 0.3 * b, -0.7 * b):
        assert abs(hz(y0)) < 1e-7
    for y0 in (0.5 * (b + w), 1.4 * w):
        ref = float(bean.strip_field(np.array([y0]), w, ha)[0])
        assert abs(hz(y0) - ref) < 1e-6 * max(1.0, abs(ref))
