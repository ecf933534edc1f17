"""Thin-film magnetization (Sec. 2 of the paper), oracle form.  TEST INFRASTRUCTURE ONLY.

Discretisation (the staggered finite-difference form of the method of lines):

* Box D = [-Lx, Lx] x [-Ly, Ly], periodic through the FFT (Sec. 2.2).  Nodes
  (p, q) sit at (-Lx + p dx, -Ly + q dy), dx = 2 Lx / nx.  Arrays are indexed
  [q, p] (y slow, x fast).
* Cell (p, q) spans nodes p..p+1, q..q+1.  ``material[q, p]`` is 0 (vacuum),
  1 (superconductor, power law (3)) or 2 (filled hole, Ohm law with rho_out,
  Sec. 2.2 last paragraph).  Omega_filled = cells with material != 0.
* The stream function g lives on nodes.  A node is an *in-node* when its four
  cells are in Omega_filled; every other node belongs to the free space
  D \\ Omega_filled of iteration (11)-(12).
* Sheet current (2), j = curl-bar g, on edges: j_x at (x_p, y_{q+1/2}) is
  (g[q+1,p] - g[q,p]) / dy, j_y at (x_{p+1/2}, y_q) is -(g[q,p+1] - g[q,p]) / dx.
* Power law (3): e = (e0/jc)(|j|/jc)^(n-1) j on edges whose two cells are
  superconducting (edge jc = mean of the two cell values); e = rho_out j on
  every other edge.  |j| on an x-edge combines j_x with the mean of the four
  nearest j_y (and symmetrically on y-edges).
* Eq. (9): dh_z/dt = -(d_x e_y - d_y e_x) with backward differences, which is
  div(rho grad g) at in-nodes.

Iteration (10)-(12) with the Fourier multipliers 2/|k| (eq. (7)) and |k|/2
(eq. (12)), both zero at k = 0, on the FFT grid k = 2 pi fftfreq(n, d).  The
update (12) may carry the Gaussian filter exp(-|k|^2 sigma^2 / 2) that Sec.
2.2 applies to its spectral derivatives and also to (12) (``sigma``; the
paper's value is sqrt(dx^2 + dy^2), see ``paper_sigma``).
The staggered form leaves it off by default (sigma = 0): with unsmoothed
finite differences inside the film the filtered update cannot correct the
high-|k| part of the free-space error and the residual stalls.  The filter
only preconditions the update: the converged gdot (zero in free space, eq.
(10)) does not depend on it.  The post-processing h_z of Sec. 2.1 uses the
plain |k|/2.

Spectral form (``deriv="spectral"``, the paper's own discretisation of Sec.
2.2): every field lives on the nodes; a derivative d/dx_a is the Fourier
multiplier i k_a exp(-|k|^2 s^2 / 2), s = ``deriv_sigma`` (default the
paper's sqrt(dx^2 + dy^2)), with the Nyquist wavenumber of that axis set to
zero (an odd symbol there has no real counterpart).  j = (d_y g, -d_x g) at
the nodes; e = rho(|j|) j with the power law at nodes whose four cells are
superconducting (jc the mean of the four cells) and rho_out at every other
node; dh_z/dt = -(d_x e_y - d_y e_x) at in-nodes.  The update (12) keeps
its own filter ``sigma``, 0 by default in both forms: filtered, it stalls
here too (a cold start at g = 0 on a 64^2 disk does not reach the stop
test in 100 iterations; unfiltered it takes at most 7).
"""
import numpy as np

from .field import AppliedField

OK, NOT_CONVERGED, NOT_FINITE = 0, 1, 2


def paper_sigma(dx, dy):
    """Width of the Gaussian filter chosen in Sec. 2.2: sqrt(dx^2 + dy^2)."""
    return float(np.hypot(dx, dy))


def shift(a, axis, off):
    """Periodic neighbour: result[..., i, ...] = a[..., i + off, ...] along ``axis``."""
    return np.roll(a, -off, axis=axis)


class FilmProblem:
    """Static data of a thin-film problem plus the warm-start buffer of Sec. 2.2.

    Parameters follow the paper's dimensionless variables (Sec. 2.3): lengths
    in units of l, fields in units of jc, time in units of mu0 jc l / e0.
    """

    def __init__(self, nx, ny, Lx, Ly, material, jc_cell=None, jc0=1.0, n=19.0, e0=1.0,
                 rho_out=1.0, lam=0.7, tol=2e-4, max_inner=100, fixed_iters=0, field=None, sigma=0.0,
                 deriv="staggered", deriv_sigma=None):
        self.nx, self.ny = int(nx), int(ny)
        self.Lx, self.Ly = float(Lx), float(Ly)
        self.dx, self.dy = 2.0 * self.Lx / self.nx, 2.0 * self.Ly / self.ny
        self.material = np.asarray(material, dtype=np.uint8).reshape(self.ny, self.nx)
        jc = np.ones((self.ny, self.nx)) if jc_cell is None else np.asarray(jc_cell, dtype=np.float64)
        self.jc_cell = jc0 * jc.reshape(self.ny, self.nx)
        self.n, self.e0, self.rho_out = float(n), float(e0), float(rho_out)
        self.lam, self.tol = float(lam), float(tol)
        self.max_inner, self.fixed_iters = int(max_inner), int(fixed_iters)
        self.field = field if field is not None else AppliedField()
        if deriv not in ("staggered", "spectral"):
            raise ValueError(deriv)
        self.deriv = deriv
        # Gaussian filters, Sec. 2.2 (None: the paper's sqrt(dx^2 + dy^2)):
        # sigma of the update (12), deriv_sigma of the spectral derivatives
        self.sigma = float(paper_sigma(self.dx, self.dy) if sigma is None else sigma)
        self.deriv_sigma = float(paper_sigma(self.dx, self.dy) if deriv_sigma is None else deriv_sigma)
        self.warm = None
        self._classify()
        self._symbols()

    # ---- geometry: which nodes and edges belong to the film (Sec. 2.2) ----
    def _classify(self):
        m = self.material
        filled = m != 0
        sc = m == 1
        # node (p, q) touches cells (p-1,q-1), (p,q-1), (p-1,q), (p,q)
        self.in_node = (filled & shift(filled, 1, -1) & shift(filled, 0, -1)
                        & shift(shift(filled, 1, -1), 0, -1))
        self.out_node = ~self.in_node
        # x-edge (p, q+1/2) separates cells (p-1, q) and (p, q)
        self.sc_xedge = sc & shift(sc, 1, -1)
        self.jc_xedge = 0.5 * (self.jc_cell + shift(self.jc_cell, 1, -1))
        # y-edge (p+1/2, q) separates cells (p, q-1) and (p, q)
        self.sc_yedge = sc & shift(sc, 0, -1)
        self.jc_yedge = 0.5 * (self.jc_cell + shift(self.jc_cell, 0, -1))
        # spectral form: a node is superconducting when its four cells are,
        # with jc the mean of the four cells
        self.sc_node = sc & shift(sc, 1, -1) & shift(sc, 0, -1) & shift(shift(sc, 1, -1), 0, -1)
        jc = self.jc_cell
        self.jc_node = 0.25 * (jc + shift(jc, 1, -1) + shift(jc, 0, -1) + shift(shift(jc, 1, -1), 0, -1))

    def _symbols(self):
        """Multipliers of eqs. (7) and (12) on the FFT grid (angular wavenumbers)."""
        kx = 2.0 * np.pi * np.fft.fftfreq(self.nx, self.dx)
        ky = 2.0 * np.pi * np.fft.fftfreq(self.ny, self.dy)
        kabs = np.sqrt(kx[None, :] ** 2 + ky[:, None] ** 2)
        self.K1 = np.zeros_like(kabs)
        nz = kabs > 0
        self.K1[nz] = 2.0 / kabs[nz]          # eq. (7): 2/|k|, set to 0 at k = 0
        self.K2 = 0.5 * kabs                  # |k|/2 (0 at k = 0): h_z of Sec. 2.1
        # eq. (12) with the Gaussian smoothing of Sec. 2.2
        gauss = np.exp(-0.5 * (self.sigma * kabs) ** 2)
        self.K2s = self.K2 * gauss
        # spectral derivatives: i k_a exp(-|k|^2 s^2 / 2), Nyquist of axis a zeroed
        dgauss = np.exp(-0.5 * (self.deriv_sigma * kabs) ** 2)
        kxn = kx.copy()
        kyn = ky.copy()
        if self.nx % 2 == 0:
            kxn[self.nx // 2] = 0.0
        if self.ny % 2 == 0:
            kyn[self.ny // 2] = 0.0
        self.DX = 1j * kxn[None, :] * dgauss
        self.DY = 1j * kyn[:, None] * dgauss

    def reset_warm_start(self):
        self.warm = None


# ---------------------------------------------------------------- operators
def sheet_current(prob, g):
    """Eq. (2): j_x = d_y g, j_y = -d_x g, forward differences onto edges."""
    jx = (shift(g, 0, 1) - g) / prob.dy
    jy = -(shift(g, 1, 1) - g) / prob.dx
    return jx, jy


def current_magnitude(jx, jy):
    """|j| on x-edges and y-edges: own component plus the mean of the 4 nearest
    components of the other orientation (the edges are staggered)."""
    # y-edges nearest to x-edge (p, q+1/2): (p-1/2, q), (p+1/2, q), (p-1/2, q+1), (p+1/2, q+1)
    jy_at_x = 0.25 * (shift(jy, 1, -1) + jy + shift(shift(jy, 1, -1), 0, 1) + shift(jy, 0, 1))
    # x-edges nearest to y-edge (p+1/2, q): (p, q-1/2), (p, q+1/2), (p+1, q-1/2), (p+1, q+1/2)
    jx_at_y = 0.25 * (shift(jx, 0, -1) + jx + shift(shift(jx, 0, -1), 1, 1) + shift(jx, 1, 1))
    sx = np.sqrt(jx ** 2 + jy_at_x ** 2)
    sy = np.sqrt(jy ** 2 + jx_at_y ** 2)
    return sx, sy


def resistivity(prob, s, jc_edge, sc_edge):
    """Power law (3): rho(|j|) = (e0/jc)(|j|/jc)^(n-1) on superconducting edges,
    rho_out (Ohm law, Sec. 2.2) elsewhere."""
    rho_pl = (prob.e0 / jc_edge) * (s / jc_edge) ** (prob.n - 1.0)
    return np.where(sc_edge, rho_pl, prob.rho_out)


def electric_field(prob, g):
    jx, jy = sheet_current(prob, g)
    sx, sy = current_magnitude(jx, jy)
    ex = resistivity(prob, sx, prob.jc_xedge, prob.sc_xedge) * jx
    ey = resistivity(prob, sy, prob.jc_yedge, prob.sc_yedge) * jy
    return ex, ey


def hdot_in(prob, g):
    """Eq. (4) in the form (9): dh_z/dt = -(d_x e_y - d_y e_x), backward
    differences from edges back to nodes (spectral derivatives in the
    spectral form).  Meaningful at in-nodes only."""
    if prob.deriv == "spectral":
        return hdot_in_spectral(prob, g)
    ex, ey = electric_field(prob, g)
    curl_e = (ey - shift(ey, 1, -1)) / prob.dx - (ex - shift(ex, 0, -1)) / prob.dy
    return -curl_e


def spectral_derivative(f, D):
    """F^{-1}[D F(f)] for a derivative symbol D (Sec. 2.2, spectral form)."""
    return np.fft.ifft2(D * np.fft.fft2(f)).real


def sheet_current_nodes(prob, g):
    """Eq. (2) at the nodes with spectral derivatives: j_x = d_y g, j_y = -d_x g."""
    return spectral_derivative(g, prob.DY), -spectral_derivative(g, prob.DX)


def hdot_in_spectral(prob, g):
    """Eq. (4) with every field at the nodes (the paper's discretisation):
    e = rho(|j|) j, the power law at superconducting nodes and rho_out at the
    others, then dh_z/dt = -(d_x e_y - d_y e_x)."""
    jx, jy = sheet_current_nodes(prob, g)
    s = np.sqrt(jx ** 2 + jy ** 2)
    rho = resistivity(prob, s, prob.jc_node, prob.sc_node)
    ex, ey = rho * jx, rho * jy
    return -(spectral_derivative(ey, prob.DX) - spectral_derivative(ex, prob.DY))


def apply_multiplier(f, K):
    """F^{-1}[K F(f)] with the discrete transform (Sec. 2.2)."""
    return np.fft.ifft2(K * np.fft.fft2(f)).real


# ------------------------------------------------------------- the RHS
def rhs(prob, g, t):
    """Right-hand side f(g, t) of the method of lines, Sec. 2.2.

    Returns (gdot, n_iterations, status).  The iteration follows the paper:
    dh/dt is known in the film from (9); in free space it is found by
    iterating (11) and the relaxed update (12), each followed by the constant
    shift A that enforces (10).  The initial free-space guess is the previous
    call's converged value (Sec. 2.2, relaxation paragraph); the very first
    call starts from dh_e/dt.  The loop stops when the mean of |gdot| over
    free-space nodes falls below tol * max(|dh_e/dt|, 1) (Sec. 2.3).  When
    ``fixed_iters`` > 0 exactly that many evaluations of (11) are done and the
    last one is returned without a stop test.  Failure to converge within
    ``max_inner`` evaluations returns status NOT_CONVERGED and clears the
    warm start (Sec. 2.2: the integrator then shrinks its step); so does a
    fixed-count evaluation whose residual is not finite (status NOT_FINITE).
    """
    hde = float(prob.field.hdot(t)[2])
    out = prob.out_node
    nout = int(out.sum())
    H = np.array(hdot_in(prob, g))
    H[out] = hde if prob.warm is None else prob.warm[out]
    # constant shift A^0 so that (10) holds: sum over D of (H - dh_e) = 0
    H[out] -= (H - hde).sum() / nout
    thr = prob.tol * max(abs(hde), 1.0)
    fixed = prob.fixed_iters > 0
    kmax = prob.fixed_iters if fixed else prob.max_inner
    for i in range(kmax):
        G = apply_multiplier(H - hde, prob.K1)              # (11) before the shift
        C = G[out].mean()                                    # makes the free-space integral vanish
        gdot = G - C
        r = np.abs(gdot[out]).mean()
        stop = (i == kmax - 1) if fixed else (r < thr)
        if stop:
            if not np.isfinite(r):
                # a failed evaluation (overflow in a stage): the integrator
                # cuts the step (Sec. 2.2) and the next call starts cold
                prob.warm = None
                return None, i + 1, NOT_FINITE
            prob.warm = H.copy()
            return gdot, i + 1, OK
        U = np.where(out, gdot, 0.0)                         # gdot_out of (12)
        V = apply_multiplier(U, prob.K2s)
        H[out] -= prob.lam * V[out]                          # relaxed, smoothed update (12)
        H[out] -= (H - hde).sum() / nout                     # A^i restores (10)
    prob.warm = None
    return None, kmax, NOT_CONVERGED


# ------------------------------------------------------------- observables
def observe(prob, g, t):
    """Post-processing of Sec. 2.1: h_z = h_e + F^{-1}[|k|/2 F(g)] on nodes,
    j from (2) on edges, and the moment m_z = sum g dx dy (the integral of g,
    equal to (1/2) int (x j_y - y j_x) because g vanishes outside the film)."""
    he = float(prob.field.h(t)[2])
    hz = he + apply_multiplier(g, prob.K2)
    jx, jy = sheet_current_nodes(prob, g) if prob.deriv == "spectral" else sheet_current(prob, g)
    mz = g.sum() * prob.dx * prob.dy
    return hz, (jx, jy), mz
