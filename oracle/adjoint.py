"""Vector-Jacobian products of the right-hand side, oracle form.  TEST
INFRASTRUCTURE ONLY.  Film (Sec. 2) below; bulk (Sec. 3) at the end of the
module.

The film right-hand side f(g, t) of Sec. 2.2 is the composition

    g  --curl-bar (2)-->  j  --power law (3)-->  e  --minus curl, eq. (9)-->  dh_in
       --iteration (10)-(12) on the free space-->  gdot.

Writing x = dh - dh_e on all nodes, the iteration is linear in x:

    start    x_out <- (warm start) ;  x <- S x
    repeat   gdot = Q x ;  x <- S (x - lam P_out K2 P_out Q x)

with Q = (I - 1 m_out^T) K1 (eq. (11) and the constant C that removes the
free-space mean of gdot), P_out the free-space mask, K1 = F^{-1} 2/|k| F and
K2 = F^{-1} |k|/2 exp(-|k|^2 sigma^2/2) F (the smoothed multiplier of (12);
real symmetric operators), m_out = 1_out / #out, and
S = I - 1_out 1^T / #out the shift A of (10) that makes sum_D x = 0.  The
warm start and dh_e only add constants, so the derivative of k evaluations of
(11) with k - 1 updates (12) in between is

    d gdot = Q B^(k-1) S E_in d(dh_in),   B = S (I - lam P_out K2 P_out Q),

and its transpose applied to a cotangent y_bar is

    x_bar = E_in^T S^T (B^T)^(k-1) Q^T y_bar,
    B^T = (I - lam Q^T P_out K2 P_out) S^T,
    Q^T z = K1 (z - m_out sum_D z),   S^T z = z - 1 (mean of z over free space).

B^T leaves the film part of its argument untouched except for the
accumulation coming from the free space, and its free-space part decays like
the forward iteration's error, so the converged (fixed-point) adjoint is the
same recursion run until the free-space part is negligible.

The film part of x_bar is then pulled back through eq. (9), the power law and
eq. (2), and through the edge jc = mean of the two cells to the per-cell map
(staggered form), or through the node quantities of the spectral form and the
node jc = mean of the four cells (film_spectral_vjp).
"""
import numpy as np

from . import film
from .film import shift

OK, NOT_CONVERGED = 0, 1


def _edge_partials(prob, g):
    """Per edge: the current, its magnitude, e, de/dj_own and de/d(other-mean)
    (the mean of the 4 nearest other-orientation components inside |j|)."""
    jx, jy = film.sheet_current(prob, g)
    jy_at_x = 0.25 * (shift(jy, 1, -1) + jy + shift(shift(jy, 1, -1), 0, 1) + shift(jy, 0, 1))
    jx_at_y = 0.25 * (shift(jx, 0, -1) + jx + shift(shift(jx, 0, -1), 1, 1) + shift(jx, 1, 1))
    out = []
    for j, oth, jce, sc in ((jx, jy_at_x, prob.jc_xedge, prob.sc_xedge),
                            (jy, jx_at_y, prob.jc_yedge, prob.sc_yedge)):
        s = np.sqrt(j ** 2 + oth ** 2)
        nm1 = prob.n - 1.0
        rho_pl = (prob.e0 / jce) * (s / jce) ** nm1
        pos = s > 0
        s2 = np.where(pos, s * s, 1.0)
        # e = rho(s) j with rho(s) = (e0/jc)(s/jc)^(n-1):
        #   de/dj   = rho + j rho'(s) j/s = rho (1 + (n-1) j^2 / s^2)
        #   de/doth = j rho'(s) oth/s    = rho (n-1) j oth / s^2
        #   de/djc  = -n e / jc
        a_pl = np.where(pos, rho_pl * (1.0 + nm1 * j * j / s2), (prob.e0 / jce) if nm1 == 0 else 0.0)
        b_pl = np.where(pos, rho_pl * nm1 * j * oth / s2, 0.0)
        e = np.where(sc, rho_pl * j, prob.rho_out * j)
        a = np.where(sc, a_pl, prob.rho_out)
        b = np.where(sc, b_pl, 0.0)
        c = np.where(sc, -prob.n * e / jce, 0.0)
        out.append((e, a, b, c))
    return out


def film_stencil_vjp(prob, g, hbar):
    """Transpose of g -> dh_in (eqs. (2), (3), (9)) applied to hbar (zero off the
    film).  Returns (g_bar, jc_cell_bar)."""
    (ex, ax, bx, cx), (ey, ay, by, cy) = _edge_partials(prob, g)
    dx, dy = prob.dx, prob.dy
    # dh(p,q) = -[(e_y(p,q) - e_y(p-1,q))/dx - (e_x(p,q) - e_x(p,q-1))/dy]
    ebar_y = (shift(hbar, 1, 1) - hbar) / dx
    ebar_x = (hbar - shift(hbar, 0, 1)) / dy
    # own-component and neighbour-mean parts of the power law
    Bx = bx * ebar_x            # cotangent of jy_at_x on x-edges
    By = by * ebar_y            # cotangent of jx_at_y on y-edges
    jbar_x = ax * ebar_x + 0.25 * (By + shift(By, 0, 1) + shift(By, 1, -1) + shift(shift(By, 1, -1), 0, 1))
    jbar_y = ay * ebar_y + 0.25 * (Bx + shift(Bx, 1, 1) + shift(Bx, 0, -1) + shift(shift(Bx, 1, 1), 0, -1))
    # j_x(p,q) = (g(p,q+1) - g(p,q))/dy, j_y(p,q) = -(g(p+1,q) - g(p,q))/dx
    gbar = (shift(jbar_x, 0, -1) - jbar_x) / dy + (jbar_y - shift(jbar_y, 1, -1)) / dx
    # edge jc = mean of its two cells: x-edge (p,q) <- cells (p,q), (p-1,q); y-edge <- (p,q), (p,q-1)
    Cx = cx * ebar_x
    Cy = cy * ebar_y
    jcbar = 0.5 * (Cx + shift(Cx, 1, 1)) + 0.5 * (Cy + shift(Cy, 0, 1))
    return gbar, jcbar


def film_spectral_vjp(prob, g, hbar):
    """Transpose of g -> dh_in in the spectral form of Sec. 2.2 applied to
    hbar (zero off the film).  Returns (g_bar, jc_cell_bar).

    The forward: j = (D_y g, -D_x g) at the nodes, e = rho(|j|) j, dh_in =
    -(D_x e_y - D_y e_x).  A filtered derivative D_a has the symbol
    i k_a exp(-|k|^2 s^2 / 2), odd and imaginary, so as a real operator its
    transpose is -D_a.  At power-law nodes de/dj = rho I + rho (n-1) j j^T / |j|^2
    and de/djc = -n e / jc; elsewhere e = rho_out j.  The node jc is the mean of
    the node's four cells."""
    jx, jy = film.sheet_current_nodes(prob, g)
    s = np.sqrt(jx ** 2 + jy ** 2)
    nm1 = prob.n - 1.0
    jce = prob.jc_node
    rho_pl = (prob.e0 / jce) * (s / jce) ** nm1
    sd = film.spectral_derivative
    # dh_in = D_y e_x - D_x e_y
    ebar_x = -sd(hbar, prob.DY)
    ebar_y = sd(hbar, prob.DX)
    jdot = jx * ebar_x + jy * ebar_y
    pos = s > 0
    fac = np.where(pos, rho_pl * nm1 * jdot / np.where(pos, s * s, 1.0), 0.0)
    sc = prob.sc_node
    jbar_x = np.where(sc, rho_pl * ebar_x + fac * jx, prob.rho_out * ebar_x)
    jbar_y = np.where(sc, rho_pl * ebar_y + fac * jy, prob.rho_out * ebar_y)
    # j_x = D_y g, j_y = -D_x g
    gbar = -sd(jbar_x, prob.DY) + sd(jbar_y, prob.DX)
    # node (p, q) takes the mean jc of cells (p,q), (p-1,q), (p,q-1), (p-1,q-1),
    # so cell (p, q) collects a quarter of nodes (p,q), (p+1,q), (p,q+1), (p+1,q+1)
    cnode = np.where(sc, -prob.n * rho_pl * jdot / jce, 0.0)
    jcbar = 0.25 * (cnode + shift(cnode, 1, 1) + shift(cnode, 0, 1) + shift(shift(cnode, 1, 1), 0, 1))
    return gbar, jcbar


def film_iteration_vjp(prob, ybar, k=None):
    """x_bar on the film nodes for the cotangent ybar of gdot.

    k = number of evaluations of (11) in the forward (fixed-count form, the
    exact transpose).  k = None: the converged form, B^T applied until the
    mean free-space |S^T mu| is below prob.tol times the mean |Q^T ybar|, at most
    prob.max_inner - 1 times.  Returns (xbar_in, count, status), count = the
    number of evaluations of (11) the transposed recursion corresponds to."""
    out = prob.out_node
    nout = int(out.sum())
    lam = prob.lam

    def QT(z):
        z = np.array(z, dtype=np.float64)
        z[out] -= z.sum() / nout
        return film.apply_multiplier(z, prob.K1)

    def ST(z):
        return z - z[out].mean()

    mu = QT(ybar)
    scale = np.abs(mu).mean()
    steps = 0
    status = OK
    if k is not None:
        for _ in range(k - 1):
            nu = ST(mu)
            w = film.apply_multiplier(np.where(out, nu, 0.0), prob.K2s)
            mu = nu - lam * QT(np.where(out, w, 0.0))
            steps += 1
    else:
        while True:
            nu = ST(mu)
            if np.abs(nu[out]).mean() < prob.tol * scale:
                break
            if steps >= prob.max_inner - 1:
                status = NOT_CONVERGED
                break
            w = film.apply_multiplier(np.where(out, nu, 0.0), prob.K2s)
            mu = nu - lam * QT(np.where(out, w, 0.0))
            steps += 1
    xbar = ST(mu)
    return np.where(prob.in_node, xbar, 0.0), steps + 1, status


def film_rhs_vjp(prob, g, t, ybar, jc0=1.0):
    """(g_bar, jc_map_bar, count, status) for the cotangent ybar of f(g, t).

    With prob.fixed_iters > 0 the forward is that many evaluations of (11) and
    this is its exact transpose; otherwise the converged form above.  The
    cell jc is jc0 times the map, so jc_map_bar = jc0 * (cotangent of the cell jc).
    t does not enter: dh_e/dt only shifts the iteration by constants."""
    k = prob.fixed_iters if prob.fixed_iters > 0 else None
    hbar, count, status = film_iteration_vjp(prob, ybar, k)
    if prob.deriv == "spectral":
        gbar, jcbar = film_spectral_vjp(prob, g, hbar)
    else:
        gbar, jcbar = film_stencil_vjp(prob, g, hbar)
    return gbar, jc0 * jcbar, count, status


# ------------------------------------------------------------------ time stepping
def bs23_step_vjp(f, fvjp, t, y, h, ybar_new):
    """Transpose of one Bogacki-Shampine step with a frozen step size h
    (the step-size controller is treated as constant):

        k1 = f(t, y),  k2 = f(t + h/2, y + h/2 k1),  k3 = f(t + 3h/4, y + 3h/4 k2)
        y_new = y + h (2/9 k1 + 1/3 k2 + 4/9 k3)

    f(t, y) -> value; fvjp(t, y, w) -> (y_bar, p_bar), the VJP of f at (t, y)
    for the state and for a parameter vector.  Returns (y_bar, p_bar)."""
    from .bs23 import A21, A32, B1, B2, B3, C2, C3
    k1 = f(t, y)
    y2 = y + (A21 * h) * k1
    k2 = f(t + C2 * h, y2)
    y3 = y + (A32 * h) * k2
    kb1 = (h * B1) * ybar_new
    kb2 = (h * B2) * ybar_new
    kb3 = (h * B3) * ybar_new
    yb3, pb3 = fvjp(t + C3 * h, y3, kb3)
    kb2 = kb2 + (A32 * h) * yb3
    yb2, pb2 = fvjp(t + C2 * h, y2, kb2)
    kb1 = kb1 + (A21 * h) * yb2
    yb1, pb1 = fvjp(t, y, kb1)
    return ybar_new + yb3 + yb2 + yb1, pb3 + pb2 + pb1


def film_pure_rhs(prob):
    """f and its VJP for a film problem with every right-hand side started
    from dh_e (no warm start), which makes f a function of (t, g) alone."""
    def f(t, y):
        prob.reset_warm_start()
        v, it, st = film.rhs(prob, y, t)
        if st != 0:
            raise RuntimeError("right-hand side did not converge")
        return v

    def fvjp(t, y, w):
        gb, jb, cnt, st = film_rhs_vjp(prob, y, t, w)
        if st != 0:
            raise RuntimeError("transposed iteration did not converge")
        return gb, jb

    return f, fvjp


def film_trajectory_grad(prob, g0, t0, steps, obs_bar):
    """Gradient of a loss on a replayed trajectory (fixed steps ``steps`` from
    t0, every right-hand side started from dh_e).  obs_bar[i] is the cotangent
    of the state after step i (None for no contribution).  Returns
    (g0_bar, jc_map_bar, final state)."""
    f, fvjp = film_pure_rhs(prob)
    from .bs23 import A21, A32, B1, B2, B3, C2, C3
    ys, ts = [np.array(g0, dtype=np.float64)], [float(t0)]
    for h in steps:
        y, t = ys[-1], ts[-1]
        k1 = f(t, y)
        k2 = f(t + C2 * h, y + (A21 * h) * k1)
        k3 = f(t + C3 * h, y + (A32 * h) * k2)
        ys.append(y + h * (B1 * k1 + B2 * k2 + B3 * k3))
        ts.append(t + h)
    ybar = np.zeros_like(ys[0])
    pbar = np.zeros_like(ys[0])
    for i in range(len(steps) - 1, -1, -1):
        if obs_bar[i] is not None:
            ybar = ybar + obs_bar[i]
        ybar, pb = bs23_step_vjp(f, fvjp, ts[i], ys[i], steps[i], ybar)
        pbar = pbar + pb
    return ybar, pbar, ys[-1]


def film_hz_vjp(prob, hz_bar):
    """Transpose of g -> h_z = h_e + F^{-1}[|k|/2 F(g)] (Sec. 2.1): the
    multiplier is real and even, so the operator is symmetric."""
    return film.apply_multiplier(hz_bar, prob.K2)


# ------------------------------------------------------------------ bulk (Sec. 3)
# The bulk right-hand side of Sec. 3.1 is the composition
#
#     h  --C (Ampere)-->  j  --power law (13)-->  e  --(-C^T), eq. (14)-->  dh_in
#        --iteration (18) on the free space-->  dh.
#
# Iteration (18) updates only the free-space edges: with H^i = dh^i,
#     H^{i+1}_out = dh_e + P_out Phi M_in C H^i,     H_in fixed,
# (M_in: mask to inside faces, Phi the Biot-Savart operator of (16)-(17)),
# so with A = P_out Phi M_in C and a fixed count k started from a constant
# warm start W, the result is
#     dh = E_in H_in + E_out H_out^k,   H_out^k = A_oo^k W + sum_{m<k} A_oo^m (A_oi H_in + dh_e),
# and its transpose applied to a cotangent y_bar is
#     H_in_bar = y_bar_in + A_oi^T s,   s = sum_{m<k} (A_oo^T)^m y_bar_out,
#     A^T = C^T M_in Phi^T P_out.
# Phi^T has the conjugate-transposed symbol of Phi.  H_in_bar is then pulled
# back through (14), the power law and Ampere's law, and through the face jc
# = mean of its two cells to the per-cell map.

def bulk_phi_t(prob, w):
    """Transpose of bulk.phi: the 3x3 symbol of Phi conjugated and transposed."""
    W = [np.fft.fftn(w[c]) for c in range(3)]
    dm, inv = prob.dminus, prob.inv_k2
    cdm = [np.conj(d) for d in dm]
    # Phi symbol rows: x <- (dy Fz - dz Fy), y <- (dz Fx - dx Fz), z <- (dx Fy - dy Fx); times inv.
    # Transpose-conjugate: component b of the result collects conj(M[a][b]) W_a.
    P = [(cdm[2] * W[1] - cdm[1] * W[2]) * inv,       # b = x: M[y][x] = dz, M[z][x] = -dy
         (-cdm[2] * W[0] + cdm[0] * W[2]) * inv,      # b = y: M[x][y] = -dz, M[z][y] = dx
         (cdm[1] * W[0] - cdm[0] * W[1]) * inv]       # b = z: M[x][z] = dy, M[y][z] = -dx
    return np.stack([np.fft.ifftn(p).real for p in P])


def _avg4_t(g, a, b):
    """Transpose of bulk._avg4(., a, b)."""
    return 0.25 * (shift(g, a, 1) + g + shift(shift(g, a, 1), b, -1) + shift(g, b, -1))


def bulk_stencil_vjp(prob, h, hbar):
    """Transpose of h -> dh_in = -C^T e(C h) applied to hbar (zero off the
    inside edges).  Returns (h_bar, jc_cell_bar)."""
    from . import bulk
    AX = bulk.AXIS
    j = bulk.curl(prob, h)
    # e_a = rho(s_a) j_a, s_a^2 = j_a^2 + sum_{b != a} avg4(j_b, a, b)^2
    avg = {}
    s = []
    for a in range(3):
        acc = j[a] ** 2
        for b in range(3):
            if b != a:
                avg[(a, b)] = bulk._avg4(j[b], AX[a], AX[b])
                acc = acc + avg[(a, b)] ** 2
        s.append(np.sqrt(acc))
    nm1 = prob.n - 1.0
    # cotangent of e: d(dh_in) = -C^T de  ->  e_bar = -C hbar
    ebar = -bulk.curl(prob, hbar)
    jbar = np.zeros_like(j)
    jcf_bar = np.zeros_like(j)
    for a in range(3):
        jce = prob.jc_face[a]
        sc = prob.sc_face[a]
        sa = s[a]
        pos = sa > 0
        s2 = np.where(pos, sa * sa, 1.0)
        rho_pl = (prob.e0 / jce) * (sa / jce) ** nm1
        rho = np.where(sc, rho_pl, prob.rho_out)
        # de_a/dj_a = rho (1 + (n-1) j_a^2 / s^2); de_a/d avg_b = rho (n-1) j_a avg_b / s^2 (power law only)
        fac = np.where(sc & pos, rho_pl * nm1 / s2, 0.0)
        jbar[a] += ebar[a] * (rho + fac * j[a] * j[a])
        for b in range(3):
            if b != a:
                jbar[b] += _avg4_t(ebar[a] * fac * j[a] * avg[(a, b)], AX[a], AX[b])
        # de_a/djc_face = -n e_a / jc (superconducting faces)
        e_pl = rho_pl * j[a]
        jcf_bar[a] = np.where(sc, ebar[a] * (-prob.n * e_pl / jce), 0.0)
    hb = bulk.curl_t(prob, jbar)
    # face jc = mean of the two cells: an a-face at (p,q,r) joins cells (p,q,r) and (p,q,r) - e_a
    jc_bar = np.zeros(prob.shape)
    for a in range(3):
        jc_bar += 0.5 * (jcf_bar[a] + shift(jcf_bar[a], AX[a], 1))
    return hb, jc_bar


def bulk_iteration_vjp(prob, ybar, k):
    """H_in_bar of the fixed-count iteration (18) (k updates) for the cotangent
    ybar of dh (all edges).  Returns H_in_bar on inside edges (0 elsewhere)."""
    from . import bulk
    ie, oe = prob.in_edge, prob.out_edge
    mu = np.where(oe, ybar, 0.0)
    s = np.zeros_like(ybar)
    nu = mu
    for m in range(k):
        s = s + nu
        if m < k - 1:
            nu = np.where(oe, bulk.curl_t(prob, prob.in_face * bulk_phi_t(prob, np.where(oe, nu, 0.0))), 0.0)
    hin_bar = np.where(ie, ybar, 0.0) + np.where(ie, bulk.curl_t(prob, prob.in_face * bulk_phi_t(prob, np.where(oe, s, 0.0))), 0.0)
    return hin_bar


def bulk_rhs_vjp(prob, h, t, ybar, jc0=1.0):
    """(h_bar, jc_map_bar) for the cotangent ybar of the fixed-count bulk
    right-hand side (prob.fixed_iters updates of (18); the warm start and
    dh_e are constants)."""
    k = prob.fixed_iters
    if k <= 0:
        raise ValueError("the bulk VJP is the transpose of a fixed inner count")
    hin_bar = bulk_iteration_vjp(prob, ybar, k)
    hb, jcb = bulk_stencil_vjp(prob, h, hin_bar)
    return hb, jc0 * jcb
