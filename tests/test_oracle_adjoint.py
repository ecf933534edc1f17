"""Pins of the oracle's vector-Jacobian products (oracle/adjoint.py) against
the oracle's forward right-hand side, which is pinned on its own: dot-product
tests <w, J v> = <J^T w, v> with J v from central differences, and a dense
Jacobian assembled column by column where the map is affine."""
import numpy as np
import pytest

from oracle import adjoint, film
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
