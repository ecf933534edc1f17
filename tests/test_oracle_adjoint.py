"""Pins of the oracle's vector-Jacobian products (oracle/adjoint.py) against
the oracle's forward right-hand side, which is pinned on its own: dot-product
tests <w, J v> = <J^T w, v> with J v from central differences, and a dense
Jacobian assembled column by column where the map is affine.  Film (Sec. 2)
and bulk (Sec. 3)."""
import numpy as np
import pytest

from oracle import adjoint, bulk, film
from oracle.field import AppliedField
from paper_1801_04869_amd import workloads as W
from tests._cases import film_case, make_oracle


def _f(prob, g, t=0.1):
    prob.reset_warm_start()
    out, it, st = film.rhs(prob, g, t)
    assert st == 0
    return out


@pytest.mark.parametrize("kind,fixed", [("offrect", 3), ("ring", 2), ("rect", 1)])
def test_film_vjp_dot_product_fixed_count(kind, fixed):
    """Fixed number of evaluations of (11): the VJP is the exact transpose of
    the composed map; central differences agree to O(eps^2)."""
    case = film_case(32, 32, kind=kind, jc_s=0.2, n=5.0, rho_out=3.0)
    prob = make_oracle(case, fixed=fixed)
    g = case["state"]
    rng = np.random.default_rng(11)
    v = rng.standard_normal(g.shape)
    w = rng.standard_normal(g.shape)
    eps = 1e-6
    Jv = (_f(prob, g + eps * v) - _f(prob, g - eps * v)) / (2 * eps)
    gbar, jcbar, cnt, st = adjoint.film_rhs_vjp(prob, g, 0.1, w)
    assert st == 0 and cnt == fixed
    lhs, rhs = np.vdot(w, Jv), np.vdot(gbar, v)
    assert abs(lhs - rhs) < 1e-6 * abs(lhs)
    # jc map direction
    jc = case["jc"]
    u = rng.standard_normal(jc.shape)

    def fj(m):
        c2 = dict(case)
        c2["jc"] = m
        return _f(make_oracle(c2, fixed=fixed), g)

    Ju = (fj(jc + eps * u) - fj(jc - eps * u)) / (2 * eps)
    lhs, rhs = np.vdot(w, Ju), np.vdot(jcbar, u)
    assert abs(lhs - rhs) < 1e-6 * abs(lhs)


@pytest.mark.parametrize("kind,fixed,nx,ny", [("offrect", 3, 32, 32), ("ring", 2, 32, 32), ("hole", 2, 48, 32)])
def test_film_spectral_vjp_dot_product_fixed_count(kind, fixed, nx, ny):
    """The spectral form (Sec. 2.2): central differences of the forward map in
    the state and in the jc map against the transposed spectral passes."""
    L = (2.25, 1.5) if kind == "hole" else (2.0, 2.0)
    case = film_case(nx, ny, L=L, kind=kind, jc_s=0.2, n=5.0, rho_out=3.0)
    prob = make_oracle(case, fixed=fixed, deriv="spectral")
    g = case["state"]
    rng = np.random.default_rng(13)
    v = rng.standard_normal(g.shape)
    w = rng.standard_normal(g.shape)
    eps = 1e-6
    Jv = (_f(prob, g + eps * v) - _f(prob, g - eps * v)) / (2 * eps)
    gbar, jcbar, cnt, st = adjoint.film_rhs_vjp(prob, g, 0.1, w)
    assert st == 0 and cnt == fixed
    lhs, rhs = np.vdot(w, Jv), np.vdot(gbar, v)
    assert abs(lhs - rhs) < 1e-6 * abs(lhs)
    jc = case["jc"]
    u = rng.standard_normal(jc.shape)

    def fj(m):
        c2 = dict(case)
        c2["jc"] = m
        return _f(make_oracle(c2, fixed=fixed, deriv="spectral"), g)

    Ju = (fj(jc + eps * u) - fj(jc - eps * u)) / (2 * eps)
    lhs, rhs = np.vdot(w, Ju), np.vdot(jcbar, u)
    assert abs(lhs - rhs) < 1e-6 * abs(lhs)


def test_film_spectral_vjp_dense_jacobian_ohmic():
    """n = 1 in the spectral form: f is affine in g, so unit-vector differences
    give the Jacobian exactly; J^T w must match the VJP."""
    case = film_case(16, 16, kind="offrect", jc_s=0.3, n=1.0, rho_out=2.0)
    prob = make_oracle(case, fixed=3, deriv="spectral")
    g = case["state"]
    f0 = _f(prob, g)
    N = g.size
    J = np.empty((N, N))
    for i in range(N):
        e = np.zeros(N)
        e[i] = 1.0
        J[:, i] = (_f(prob, g + e.reshape(g.shape)) - f0).ravel()
    w = np.random.default_rng(4).standard_normal(g.shape)
    gbar, _, _, _ = adjoint.film_rhs_vjp(prob, g, 0.1, w)
    ref = (J.T @ w.ravel()).reshape(g.shape)
    assert np.abs(gbar - ref).max() < 1e-10 * np.abs(ref).max()


def test_film_vjp_dense_jacobian_ohmic():
    """n = 1 (Ohm law in the film): f is affine in g, so unit-vector
    differences give the Jacobian exactly; J^T w must match the VJP."""
    case = film_case(16, 16, kind="offrect", jc_s=0.3, n=1.0, rho_out=2.0)
    prob = make_oracle(case, fixed=4)
    g = case["state"]
    f0 = _f(prob, g)
    N = g.size
    J = np.empty((N, N))
    for i in range(N):
        e = np.zeros(N)
        e[i] = 1.0
        J[:, i] = (_f(prob, g + e.reshape(g.shape)) - f0).ravel()
    w = np.random.default_rng(2).standard_normal(g.shape)
    gbar, _, _, _ = adjoint.film_rhs_vjp(prob, g, 0.1, w)
    ref = (J.T @ w.ravel()).reshape(g.shape)
    assert np.abs(gbar - ref).max() < 1e-10 * np.abs(ref).max()


def test_film_vjp_converged_fixed_point():
    """Converged form: the transposed recursion run to its own stop test is the
    derivative of the converged map (both at a tight tolerance)."""
    case = film_case(32, 32, kind="rect", jc_s=0.1, n=4.0)
    prob = make_oracle(case, tol=1e-13, max_inner=5000)
    g = case["state"]
    rng = np.random.default_rng(5)
    v = rng.standard_normal(g.shape)
    w = rng.standard_normal(g.shape)
    eps = 1e-5
    Jv = (_f(prob, g + eps * v) - _f(prob, g - eps * v)) / (2 * eps)
    gbar, jcbar, cnt, st = adjoint.film_rhs_vjp(prob, g, 0.1, w)
    assert st == 0 and cnt > 5
    lhs, rhs = np.vdot(w, Jv), np.vdot(gbar, v)
    assert abs(lhs - rhs) < 1e-6 * abs(lhs)


def test_film_iteration_vjp_is_transpose_of_linear_iteration():
    """The iteration alone (dh_in -> gdot at fixed count) is linear; assemble it
    on a 16 x 8 grid from unit film inputs and compare with the transposed
    recursion, including free-space and film cotangents."""
    case = film_case(16, 8, L=(2.0, 1.0), kind="offrect")
    prob = make_oracle(case, fixed=3)
    inn = prob.in_node
    idx = np.flatnonzero(inn.ravel())
    out = prob.out_node
    nout = int(out.sum())

    def iterate(hin):
        # the forward iteration of film.rhs with dh_e = 0 and a zero warm start
        H = np.where(inn, hin, 0.0)
        H[out] -= H.sum() / nout
        for i in range(3):
            G = film.apply_multiplier(H, prob.K1)
            gdot = G - G[out].mean()
            if i == 2:
                return gdot
            V = film.apply_multiplier(np.where(out, gdot, 0.0), prob.K2)
            H[out] -= prob.lam * V[out]
            H[out] -= H.sum() / nout

    A = np.empty((inn.size, len(idx)))
    for c, i in enumerate(idx):
        e = np.zeros(inn.size)
        e[i] = 1.0
        A[:, c] = iterate(e.reshape(inn.shape)).ravel()
    y = np.random.default_rng(9).standard_normal(inn.shape)
    xbar, cnt, st = adjoint.film_iteration_vjp(prob, y, k=3)
    assert cnt == 3
    assert np.abs(xbar.ravel()[idx] - A.T @ y.ravel()).max() < 1e-12 * np.abs(A.T @ y.ravel()).max()
    assert np.all(xbar[~inn] == 0.0)


def test_bs23_step_vjp_scalar_linear():
    """For y' = a y (+ p as a source) one frozen step is y_new = R(ah) y with
    R(z) = 1 + z + z^2/2 + z^3/6 (the pair is third order); its transpose is
    the same factor."""
    from oracle.adjoint import bs23_step_vjp
    a, p = -3.0, 0.7
    f = lambda t, y: a * y + p
    fvjp = lambda t, y, w: (a * w, w)
    h = 0.1
    yb, pb = bs23_step_vjp(f, fvjp, 0.0, np.array([1.3]), h, np.array([1.0]))
    z = a * h
    assert abs(yb[0] - (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-15
    # d y_new / d p: y_new = R y + p h (1 + z/2 + z^2/6)
    assert abs(pb[0] - h * (1 + z / 2 + z * z / 6)) < 1e-15


def test_film_trajectory_gradient_finite_differences():
    """Gradient of L = <w1, y_2> + <w2, y_4> over 4 replayed BS23 steps of a
    32 x 32 film (fixed inner count, no warm start) with respect to g0 and the
    jc map, against central differences of the replayed forward."""
    case = film_case(32, 32, kind="offrect", jc_s=0.2, n=5.0, rho_out=3.0)
    prob = make_oracle(case, fixed=3)
    g0 = case["state"]
    steps = [2e-3, 3e-3, 1.5e-3, 2.5e-3]
    rng = np.random.default_rng(21)
    w1, w2 = rng.standard_normal(g0.shape), rng.standard_normal(g0.shape)
    obs_bar = [None, w1, None, w2]
    gb, jb, _ = adjoint.film_trajectory_grad(prob, g0, 0.1, steps, obs_bar)

    def loss(g, jcm):
        c2 = dict(case)
        c2["jc"] = jcm
        p2 = make_oracle(c2, fixed=3)
        f, _ = adjoint.film_pure_rhs(p2)
        from oracle.bs23 import A21, A32, B1, B2, B3, C2, C3
        y, t, L = g, 0.1, 0.0
        for i, h in enumerate(steps):
            k1 = f(t, y)
            k2 = f(t + C2 * h, y + (A21 * h) * k1)
            k3 = f(t + C3 * h, y + (A32 * h) * k2)
            y, t = y + h * (B1 * k1 + B2 * k2 + B3 * k3), t + h
            if obs_bar[i] is not None:
                L += np.vdot(obs_bar[i], y)
        return L

    v = rng.standard_normal(g0.shape)
    u = rng.standard_normal(g0.shape)
    eps = 1e-5
    jc = case["jc"]
    dL = (loss(g0 + eps * v, jc) - loss(g0 - eps * v, jc)) / (2 * eps)
    assert abs(dL - np.vdot(gb, v)) < 1e-6 * abs(dL)
    dL = (loss(g0, jc + eps * u) - loss(g0, jc - eps * u)) / (2 * eps)
    assert abs(dL - np.vdot(jb, u)) < 1e-6 * abs(dL)


# ------------------------------------------------------------------ bulk (Sec. 3)
def _bulk_prob(fixed=2, n=7.0, jc_s=0.2, rho_out=3.0, seed=4):
    nx, ny, nz = 12, 10, 8
    L = (1.5, 1.25, 1.0)
    m = W.bulk_box(nx, ny, nz, *L, 0.75, 0.6, 0.5)
    m = np.roll(m, (1, -1, 0), axis=(0, 1, 2))
    # one normal-conducting cell block inside the sample (rho_out path)
    m[3:5, 4:6, 5:7][m[3:5, 4:6, 5:7] == 1] = 2
    jc = W.lognormal_jc((nz, ny, nx), jc_s, 2.0, seed) if jc_s > 0 else None
    fld = AppliedField(kind=0, direction=(0.3, -0.2, 0.9), rate=0.7)
    p = bulk.BulkProblem(nx, ny, nz, *L, m, jc_cell=jc, n=n, rho_out=rho_out, fixed_iters=fixed, field=fld)
    he = fld.h(0.3)
    h = W.bulk_snapshot(m, 2 * L[0] / nx, he, delta=0.3, seed=seed + 1)
    rng = np.random.default_rng(seed + 2)
    h = h + 0.05 * rng.standard_normal(h.shape)
    return p, h, jc


def test_bulk_phi_transpose_dot_product():
    """<Phi j, w> = <j, Phi^T w> for random face and edge fields (the Fourier
    symbol of Phi conjugated and transposed)."""
    p, h, _ = _bulk_prob()
    rng = np.random.default_rng(11)
    j = rng.standard_normal((3,) + p.shape)
    w = rng.standard_normal((3,) + p.shape)
    lhs = np.sum(bulk.phi(p, j) * w)
    rhs = np.sum(j * adjoint.bulk_phi_t(p, w))
    assert abs(lhs - rhs) < 1e-12 * np.linalg.norm(j) * np.linalg.norm(w)


def _bulk_f(p, h, t=0.3):
    p.reset_warm_start()
    v, it, st = bulk.rhs(p, h, t)
    assert st == 0
    return v


@pytest.mark.parametrize("fixed", [1, 3])
def test_bulk_rhs_vjp_central_differences(fixed):
    """<f(h + eps v) - f(h - eps v), ybar> / (2 eps) = <v, f'(h)^T ybar> for the
    fixed-count bulk right-hand side (power law with n = 7, a normal-conducting
    block, log-normal jc), random directions v and cotangents ybar."""
    p, h, _ = _bulk_prob(fixed=fixed)
    rng = np.random.default_rng(21 + fixed)
    ybar = rng.standard_normal(h.shape)
    hb, jcb = adjoint.bulk_rhs_vjp(p, h, 0.3, ybar)
    for trial in range(2):
        v = rng.standard_normal(h.shape)
        eps = 1e-6
        fd = np.sum((_bulk_f(p, h + eps * v) - _bulk_f(p, h - eps * v)) * ybar) / (2 * eps)
        an = np.sum(v * hb)
        assert abs(fd - an) < 1e-6 * max(abs(an), np.linalg.norm(hb) * np.linalg.norm(v) * 1e-3)


def test_bulk_rhs_vjp_jc_map_central_differences():
    """The cotangent of the per-cell jc map against central differences of the
    fixed-count right-hand side in random map directions."""
    p, h, jc = _bulk_prob(fixed=2)
    rng = np.random.default_rng(31)
    ybar = rng.standard_normal(h.shape)
    hb, jcb = adjoint.bulk_rhs_vjp(p, h, 0.3, ybar)
    base = p.jc_cell.copy()
    for trial in range(2):
        d = rng.standard_normal(base.shape)
        eps = 1e-6
        vals = []
        for sgn in (1, -1):
            q, _, _ = _bulk_prob(fixed=2)
            q.jc_cell = base * (1 + sgn * eps * d)
            q._classify()
            vals.append(_bulk_f(q, h))
        fd = np.sum((vals[0] - vals[1]) * ybar) / (2 * eps)
        an = np.sum(jcb * base * d)
        assert abs(fd - an) < 1e-6 * max(abs(an), 1e-12)
