"""Bulk magnetization (Sec. 3 of the paper), oracle form.  TEST INFRASTRUCTURE ONLY.

Discretisation (staggered finite differences on a Yee lattice):

* Box D = [-Lx, Lx] x [-Ly, Ly] x [-Lz, Lz], periodic through the FFT
  (Sec. 3.1, last paragraph).  Nodes (p, q, r) at (-Lx + p dx, ...), arrays
  indexed [r, q, p] (z slowest, x fastest).
* Cell (p, q, r) spans nodes p..p+1 etc.; ``material[r, q, p]`` is 0 (free
  space), 1 (superconductor, power law (13)) or 2 (normal conductor, Ohm law
  with rho_out).
* The field h lives on edges: h_x at (x_{p+1/2}, y_q, z_r) and cyclically.
  The current j = curl h (Ampere law, Sec. 3.1) lives on faces: j_x at
  (x_p, y_{q+1/2}, z_{r+1/2}) and cyclically; the curl C uses forward
  differences and its transpose C^T (backward differences) maps face fields
  back to edges, so Faraday's law (14) reads dh/dt = -C^T e.
* A face is *in* when both of its cells are in Omega (material != 0); an
  edge is *in* when all four of its cells are.  Free space is everything else.
* Power law (13) on faces whose two cells are superconducting (face jc = mean
  of the two cells); rho_out on every other face.  |j| on an x-face combines
  j_x with the means of the four nearest j_y and the four nearest j_z.

The Biot-Savart operator Phi of eqs. (16)-(17) is applied in Fourier space.
The default is the lattice form Phi_h = C^T (-Delta_h)^{-1}: symbol
(i k x j)/|k|^2 of eq. (17) with i k_a replaced by the backward-difference
symbol (1 - exp(-i k_a d_a))/d_a and |k|^2 by sum 4 sin^2(k_a d_a / 2)/d_a^2,
so that C Phi_h j = j exactly for divergence-free lattice currents.  The
continuum symbol of eq. (17) is available as ``phi_kind='continuum'``.
Both replace 1/|k|^2 by 0 at k = 0 (Sec. 3.1).
"""
import numpy as np

from .field import AppliedField

OK, NOT_CONVERGED, NOT_FINITE = 0, 1, 2
X, Y, Z = 2, 1, 0          # array axis of each coordinate


def shift(a, axis, off):
    """Periodic neighbour: result[i] = a[i + off] along ``axis``."""
    return np.roll(a, -off, axis=axis)


class BulkProblem:
    """Static data of a bulk problem and the warm-start buffer (Sec. 3.1)."""

    def __init__(self, nx, ny, nz, Lx, Ly, Lz, material, jc_cell=None, jc0=1.0, n=25.0,
                 e0=1.0, rho_out=1.0, tol=1e-4, max_inner=100, fixed_iters=0, field=None,
                 phi_kind="lattice"):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.L = (float(Lx), float(Ly), float(Lz))
        self.dx, self.dy, self.dz = 2 * self.L[0] / self.nx, 2 * self.L[1] / self.ny, 2 * self.L[2] / self.nz
        self.d = {X: self.dx, Y: self.dy, Z: self.dz}
        shape = (self.nz, self.ny, self.nx)
        self.shape = shape
        self.material = np.asarray(material, dtype=np.uint8).reshape(shape)
        jc = np.ones(shape) if jc_cell is None else np.asarray(jc_cell, dtype=np.float64).reshape(shape)
        self.jc_cell = jc0 * jc
        self.n, self.e0, self.rho_out = float(n), float(e0), float(rho_out)
        self.tol, self.max_inner, self.fixed_iters = float(tol), int(max_inner), int(fixed_iters)
        self.field = field if field is not None else AppliedField()
        self.phi_kind = phi_kind
        self.warm = None
        self._classify()
        self._symbols()

    def _classify(self):
        m = self.material
        filled, sc = m != 0, m == 1
        axes = (X, Y, Z)
        self.in_face, self.sc_face, self.jc_face = [], [], []
        for a in axes:                     # component order x, y, z
            self.in_face.append(filled & shift(filled, a, -1))
            self.sc_face.append(sc & shift(sc, a, -1))
            self.jc_face.append(0.5 * (self.jc_cell + shift(self.jc_cell, a, -1)))
        self.in_edge = []
        for a in axes:
            b, c = [ax for ax in axes if ax != a]
            f = filled & shift(filled, b, -1) & shift(filled, c, -1) & shift(shift(filled, b, -1), c, -1)
            self.in_edge.append(f)
        self.in_face = np.stack(self.in_face)
        self.sc_face = np.stack(self.sc_face)
        self.jc_face = np.stack(self.jc_face)
        self.in_edge = np.stack(self.in_edge)
        self.out_edge = ~self.in_edge

    def _symbols(self):
        th = [2 * np.pi * np.fft.fftfreq(n) for n in (self.nx, self.ny, self.nz)]   # k_a d_a
        tx, ty, tz = np.meshgrid(th[0], th[1], th[2], indexing="xy")
        # meshgrid 'xy' with (x, y, z) returns arrays indexed [y, x, z]; reorder to [z, y, x]
        tx, ty, tz = (np.transpose(a, (2, 0, 1)) for a in (tx, ty, tz))
        if self.phi_kind == "lattice":
            dm = [(1 - np.exp(-1j * tx)) / self.dx,
                  (1 - np.exp(-1j * ty)) / self.dy,
                  (1 - np.exp(-1j * tz)) / self.dz]
            k2 = (4 * np.sin(tx / 2) ** 2 / self.dx ** 2 + 4 * np.sin(ty / 2) ** 2 / self.dy ** 2
                  + 4 * np.sin(tz / 2) ** 2 / self.dz ** 2)
        elif self.phi_kind == "continuum":
            dm = [1j * tx / self.dx, 1j * ty / self.dy, 1j * tz / self.dz]
            k2 = (tx / self.dx) ** 2 + (ty / self.dy) ** 2 + (tz / self.dz) ** 2
        else:
            raise ValueError(self.phi_kind)
        inv = np.zeros_like(k2)
        inv[k2 > 0] = 1.0 / k2[k2 > 0]      # 1/|k|^2 replaced by 0 at k = 0 (Sec. 3.1)
        self.dminus = dm
        self.inv_k2 = inv

    def reset_warm_start(self):
        self.warm = None


# ---------------------------------------------------------------- operators
def fdiff(f, prob, a):
    return (shift(f, a, 1) - f) / prob.d[a]


def bdiff(f, prob, a):
    return (f - shift(f, a, -1)) / prob.d[a]


def curl(prob, h):
    """Ampere law j = curl h (Sec. 3.1) from edges to faces: forward differences."""
    hx, hy, hz = h
    return np.stack([fdiff(hz, prob, Y) - fdiff(hy, prob, Z),
                     fdiff(hx, prob, Z) - fdiff(hz, prob, X),
                     fdiff(hy, prob, X) - fdiff(hx, prob, Y)])


def curl_t(prob, e):
    """Transpose of ``curl``: backward-difference curl from faces to edges, so
    that Faraday's law (14) reads dh/dt = -curl_t(e)."""
    ex, ey, ez = e
    return np.stack([bdiff(ez, prob, Y) - bdiff(ey, prob, Z),
                     bdiff(ex, prob, Z) - bdiff(ez, prob, X),
                     bdiff(ey, prob, X) - bdiff(ex, prob, Y)])


def _avg4(f, a, b):
    """Mean of the four b-faces nearest to an a-face: offsets {-1, 0} along
    axis a and {0, +1} along axis b."""
    return 0.25 * (shift(f, a, -1) + f + shift(shift(f, a, -1), b, 1) + shift(f, b, 1))


AXIS = (X, Y, Z)


def current_magnitude(j):
    """|j| on the faces of each orientation (staggered components averaged)."""
    s = []
    for ca in range(3):
        acc = j[ca] ** 2
        for cb in range(3):
            if cb != ca:
                acc = acc + _avg4(j[cb], AXIS[ca], AXIS[cb]) ** 2
        s.append(np.sqrt(acc))
    return np.stack(s)


def resistivity(prob, s):
    """Power law (13) on superconducting faces, rho_out elsewhere (Sec. 3.1)."""
    rho_pl = (prob.e0 / prob.jc_face) * (s / prob.jc_face) ** (prob.n - 1.0)
    return np.where(prob.sc_face, rho_pl, prob.rho_out)


def electric_field(prob, h):
    j = curl(prob, h)
    return resistivity(prob, current_magnitude(j)) * j


def hdot_in(prob, h):
    """Faraday law (14): dh/dt = -curl e; valid on in-edges."""
    return -curl_t(prob, electric_field(prob, h))


def phi(prob, j):
    """Operator Phi of eq. (16) applied through the Fourier symbol of eq. (17)
    (lattice or continuum form, see the module docstring)."""
    F = [np.fft.fftn(j[c]) for c in range(3)]
    dm, inv = prob.dminus, prob.inv_k2
    P = [(dm[1] * F[2] - dm[2] * F[1]) * inv,
         (dm[2] * F[0] - dm[0] * F[2]) * inv,
         (dm[0] * F[1] - dm[1] * F[0]) * inv]
    return np.stack([np.fft.ifftn(p).real for p in P])


# ------------------------------------------------------------- the RHS
def rhs(prob, h, t):
    """Right-hand side f(t, h) of Sec. 3.1/3.2.

    dh/dt on in-edges comes from Faraday's law; on free-space edges it is
    found by iteration (18): jdot = curl dh masked to in-faces, then the
    free-space values become dh_e/dt + Phi[jdot].  The iteration stops when
    the mean of |dh^{i+1} - dh^i| over free-space edges falls below
    tol * max(|dh_e/dt|, 1) (Sec. 3.1, last paragraph).  The first guess is
    the previous call's result (warm start, as for films) or dh_e/dt.
    ``fixed_iters`` > 0 runs exactly that many updates without a stop test.
    Returns (hdot, n_iterations, status).
    """
    hde = prob.field.hdot(t)
    ie, oe = prob.in_edge, prob.out_edge
    nout = int(oe.sum())
    H = hdot_in(prob, h)
    for c in range(3):
        H[c][oe[c]] = hde[c] if prob.warm is None else prob.warm[c][oe[c]]
    thr = prob.tol * max(np.linalg.norm(hde), 1.0)
    fixed = prob.fixed_iters > 0
    kmax = prob.fixed_iters if fixed else prob.max_inner
    for i in range(kmax):
        jdot = curl(prob, H) * prob.in_face           # jdot_in of (18)
        P = phi(prob, jdot)
        Hn = np.where(ie, H, hde[:, None, None, None] + P)
        r = np.abs(Hn - H)[oe].sum() / nout
        H = Hn
        stop = (i == kmax - 1) if fixed else (r < thr)
        if stop:
            if not np.isfinite(r):
                # a failed evaluation: no warm start for the next call (Sec. 2.2)
                prob.warm = None
                return None, i + 1, NOT_FINITE
            prob.warm = H.copy()
            return H, i + 1, OK
    prob.warm = None
    return None, kmax, NOT_CONVERGED


# ------------------------------------------------------------- observables
def face_centres(prob):
    """Coordinates of the face centres of each orientation, arrays [r, q, p]."""
    xs = [-prob.L[0] + prob.dx * np.arange(prob.nx), -prob.L[1] + prob.dy * np.arange(prob.ny),
          -prob.L[2] + prob.dz * np.arange(prob.nz)]
    half = [prob.dx / 2, prob.dy / 2, prob.dz / 2]
    out = []
    for c in range(3):     # c-face: node coordinate along c, half-shifted along the other two
        pos = [xs[a] + (0.0 if a == c else half[a]) for a in range(3)]
        Xc = pos[0][None, None, :] + 0 * pos[1][None, :, None] + 0 * pos[2][:, None, None]
        Yc = 0 * pos[0][None, None, :] + pos[1][None, :, None] + 0 * pos[2][:, None, None]
        Zc = 0 * pos[0][None, None, :] + 0 * pos[1][None, :, None] + pos[2][:, None, None]
        out.append((Xc, Yc, Zc))
    return out


def observe(prob, h, t):
    """h_z on z-edges (the state's z component), j = curl h on faces and the
    magnetic moment m = (1/2) sum r x j dV, each component of r x j summed over
    the faces that carry the current component involved; origin at the box
    centre."""
    j = curl(prob, h)
    dV = prob.dx * prob.dy * prob.dz
    (xX, yX, zX), (xY, yY, zY), (xZ, yZ, zZ) = face_centres(prob)
    m = 0.5 * dV * np.array([
        (yZ * j[2]).sum() - (zY * j[1]).sum(),
        (zX * j[0]).sum() - (xZ * j[2]).sum(),
        (xY * j[1]).sum() - (yX * j[0]).sum()])
    return h[2].copy(), j, m
