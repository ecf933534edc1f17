"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only builds *inputs*: material masks, critical-current maps,
Bean-like snapshot states and the named workload configurations.  It holds
none of the method's arithmetic (no curls, power law, Fourier multipliers or
iteration) and imports neither the HIP binding nor the oracle.

Geometry conventions (shared by both implementations): the box is
[-L, L] along each axis with n nodes at -L + i*d, d = 2L/n; cell i spans
nodes i..i+1, so its centre is at -L + (i + 1/2) d.  Material codes:
0 free space, 1 superconductor, 2 normal (Ohmic) filling.
"""
import numpy as np
from scipy import ndimage

VACUUM, SC, OHMIC = 0, 1, 2


def cell_centres(n, L):
    d = 2.0 * L / n
    return -L + (np.arange(n) + 0.5) * d


# ------------------------------------------------------------------ 2D masks
def film_rect(nx, ny, Lx, Ly, ax, ay):
    """Rectangle |x| <= ax, |y| <= ay (cells whose centres lie inside)."""
    xc, yc = cell_centres(nx, Lx), cell_centres(ny, Ly)
    m = (np.abs(xc)[None, :] < ax) & (np.abs(yc)[:, None] < ay)
    return m.astype(np.uint8) * SC


def film_disk(nx, ny, Lx, Ly, R):
    xc, yc = cell_centres(nx, Lx), cell_centres(ny, Ly)
    r2 = xc[None, :] ** 2 + yc[:, None] ** 2
    return (r2 < R * R).astype(np.uint8) * SC


def film_ring(nx, ny, Lx, Ly, r_in, r_out):
    """Annulus r_in <= r <= r_out with its hole filled by a normal conductor."""
    xc, yc = cell_centres(nx, Lx), cell_centres(ny, Ly)
    r2 = xc[None, :] ** 2 + yc[:, None] ** 2
    m = np.zeros((ny, nx), np.uint8)
    m[r2 < r_out ** 2] = SC
    m[r2 < r_in ** 2] = OHMIC
    return m


def film_rect_hole(nx, ny, Lx, Ly, ax, ay, cx, cy, r):
    """Rectangle |x| <= ax, |y| <= ay with the circular hole
    (x - cx)^2 + (y - cy)^2 <= r^2 filled by a normal conductor (the film of
    Sec. 2.3, Fig. 3: ax = 1.5, ay = 1, centre (0.5, 0.25), r = 0.5)."""
    m = film_rect(nx, ny, Lx, Ly, ax, ay)
    xc, yc = cell_centres(nx, Lx), cell_centres(ny, Ly)
    hole = (xc[None, :] - cx) ** 2 + (yc[:, None] - cy) ** 2 <= r ** 2
    m[hole & (m == SC)] = OHMIC
    return m


def film_slot(nx, ny, Lx, Ly, half, slot_cells):
    """Square |x|,|y| <= half minus the slot {x >= 0, |y| <= slot_cells*dy/2},
    open to the free space (the slot belongs to the free space)."""
    m = film_rect(nx, ny, Lx, Ly, half, half)
    xc, yc = cell_centres(nx, Lx), cell_centres(ny, Ly)
    dy = 2.0 * Ly / ny
    slot = (xc[None, :] >= 0) & (np.abs(yc)[:, None] < 0.5 * slot_cells * dy)
    m[slot] = VACUUM
    return m


# ------------------------------------------------------------------ 3D masks
def bulk_box(nx, ny, nz, Lx, Ly, Lz, ax, ay, az):
    """Cuboid |x| <= ax, |y| <= ay, |z| <= az; array indexed [z, y, x]."""
    xc, yc, zc = cell_centres(nx, Lx), cell_centres(ny, Ly), cell_centres(nz, Lz)
    m = ((np.abs(xc)[None, None, :] < ax) & (np.abs(yc)[None, :, None] < ay)
         & (np.abs(zc)[:, None, None] < az))
    return m.astype(np.uint8) * SC


def bulk_ball_shell(nx, ny, nz, L, r_in, r_out):
    xc = cell_centres(nx, L)
    yc = cell_centres(ny, L)
    zc = cell_centres(nz, L)
    r2 = xc[None, None, :] ** 2 + yc[None, :, None] ** 2 + zc[:, None, None] ** 2
    return ((r2 <= r_out ** 2) & (r2 >= r_in ** 2)).astype(np.uint8) * SC


# ------------------------------------------------------------------ jc maps
def lognormal_jc(shape, s, ell, seed, jc0=1.0):
    """Per-cell critical current jc = jc0 exp(s xi - s^2/2).

    xi is a unit-variance Gaussian random field with covariance
    exp(-r^2 / (2 ell^2)) (r in cells): white noise from numpy's PCG64(seed)
    filtered (periodically) by a Gaussian of standard deviation ell/sqrt(2)
    cells and renormalised to unit sample variance."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal(shape)
    xi = ndimage.gaussian_filter(w, sigma=ell / np.sqrt(2.0), mode="wrap")
    xi = (xi - xi.mean()) / xi.std()
    return jc0 * np.exp(s * xi - 0.5 * s * s)


# ------------------------------------------------------------------ snapshots
def film_node_inside(material):
    """Nodes whose four neighbouring cells are all non-vacuum (geometry only)."""
    f = material != 0
    return f & np.roll(f, 1, 1) & np.roll(f, 1, 0) & np.roll(np.roll(f, 1, 1), 1, 0)


def film_snapshot(material, dx, delta=0.15, jc=1.0, noise=1e-3, seed=1801):
    """Bean-like stream function for a film: g = -jc min(dist(node, boundary), delta)
    on inside nodes, 0 elsewhere, plus seeded noise of relative size ``noise``
    on inside nodes (a sand-pile profile with |grad g| = jc in a band of width
    delta; negative sign = screening an increasing field)."""
    inside = film_node_inside(material)
    dist = ndimage.distance_transform_edt(inside) * dx
    g = -jc * np.minimum(dist, delta)
    rng = np.random.Generator(np.random.PCG64(seed))
    g = g + noise * delta * rng.standard_normal(g.shape) * inside
    return np.where(inside, g, 0.0)


def bulk_snapshot(material, d, he, delta=0.2, jc=1.0, noise=1e-3, seed=1804):
    """Bean-like field for a bulk sample: h = h_e + psi z_hat with
    psi = -jc min(dist_xy(edge, boundary), delta) on z-edges whose four cells
    are all non-vacuum (0 elsewhere), plus seeded noise of size noise*jc*d on
    those edges.  Shape (3, nz, ny, nx), float64."""
    f = material != 0
    zin = f & np.roll(f, 1, 2) & np.roll(f, 1, 1) & np.roll(np.roll(f, 1, 2), 1, 1)
    nz, ny, nx = material.shape
    psi = np.zeros(material.shape)
    for r in range(nz):
        if zin[r].any():
            psi[r] = -jc * np.minimum(ndimage.distance_transform_edt(zin[r]) * d, delta)
    rng = np.random.Generator(np.random.PCG64(seed))
    psi = psi + noise * jc * d * rng.standard_normal(psi.shape) * zin
    psi = np.where(zin, psi, 0.0)
    h = np.empty((3, nz, ny, nx))
    for c in range(3):
        h[c] = he[c]
    h[2] += psi
    return h


# ------------------------------------------------------------------ workloads
def workload(name):
    """Named workload configurations (dimensionless units).

    film-128      64x64-cell square film in a 128^2 periodic grid, [-2,2]^2
    film-2048-ring / film-2048-slot   1024^2-cell ring / slotted square in 2048^2
    film-768x512-hole  rectangular film with a circular hole (Sec. 2.3, Fig. 3):
                  768x512 grid on |x| <= 2.25, |y| <= 1.5, n = 50, rho_out = 500
                  in the hole and outside, h_e = t
    bulk-64       32^3-cell cube in a 64^3 grid, [-2,2]^3, n = 25
    bulk-256      128^3-cell cube in a 256^3 grid, [-2,2]^3, n = 50, tilted field,
                  log-normal jc (s = 0.15, correlation 6 cells)
    bulk-512x512x128  256x256x64-cell cuboid in 512x512x128, n = 100, rotating field
    """
    if name == "film-128":
        return dict(dim=2, n=(128, 128), L=(2.0, 2.0), half=(1.0, 1.0), nexp=19.0,
                    field=dict(kind=0, dir=(0, 0, 1), amp=1.0, omega=1.0, rate=1.0))
    if name in ("film-2048-ring", "film-2048-slot"):
        return dict(dim=2, n=(2048, 2048), L=(2.0, 2.0), nexp=30.0, rho_out=500.0,
                    jc=dict(s=0.2, ell=8.0, seed=1801 if name.endswith("ring") else 1802),
                    field=dict(kind=1, dir=(0, 0, 1), amp=0.8, omega=1.25, rate=1.0))
    if name == "film-768x512-hole":
        # lambda: the relaxation of (12) below 2 / mu_max at this resolution
        return dict(dim=2, n=(768, 512), L=(2.25, 1.5), nexp=50.0, rho_out=500.0, lam=0.4,
                    hole=dict(ax=1.5, ay=1.0, cx=0.5, cy=0.25, r=0.5),
                    field=dict(kind=0, dir=(0, 0, 1), amp=1.0, omega=1.0, rate=1.0))
    if name == "bulk-64":
        return dict(dim=3, n=(64, 64, 64), L=(2.0, 2.0, 2.0), half=(1.0, 1.0, 1.0), nexp=25.0,
                    field=dict(kind=0, dir=(0, 0, 1), amp=1.0, omega=1.0, rate=1.0))
    if name == "bulk-256":
        a = np.deg2rad(30.0)
        return dict(dim=3, n=(256, 256, 256), L=(2.0, 2.0, 2.0), half=(1.0, 1.0, 1.0), nexp=50.0,
                    jc=dict(s=0.15, ell=6.0, seed=1803),
                    field=dict(kind=0, dir=(np.sin(a), 0.0, np.cos(a)), amp=1.0, omega=1.0, rate=1.0))
    if name == "bulk-512x512x128":
        return dict(dim=3, n=(512, 512, 128), L=(8.0, 8.0, 2.0), half=(4.0, 4.0, 1.0), nexp=100.0,
                    jc=dict(s=0.15, ell=6.0, seed=1805),
                    field=dict(kind=2, dir=(0, 0, 1), amp=1.0, omega=1.0, rate=1.0))
    raise KeyError(name)
