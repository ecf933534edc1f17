"""GPU gradients through time: the transposed BS23 step (mag_step_vjp), the
checkpointed autograd trajectory and the h_z observation, against the oracle
(oracle/adjoint.py) on replayed steps with no warm start."""
import numpy as np
import pytest

from tests._cases import film_case, make_gpu, make_oracle, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import adjoint  # noqa: E402
from paper_1801_04869_amd import api  # noqa: E402
from paper_1801_04869_amd import autograd as ag  # noqa: E402


def _case():
    return film_case(64, 64, kind="offrect", jc_s=0.2, n=5.0, rho_out=3.0)


def test_step_vjp_matches_oracle():
    case = _case()
    ctx = make_gpu(case, api.FP64, fixed=3)
    ctx.set_warm_start(False)
    prob = make_oracle(case, fixed=3)
    f, fvjp = adjoint.film_pure_rhs(prob)
    g = case["state"]
    yb = np.random.default_rng(2).standard_normal(g.shape)
    ref_y, ref_jc = adjoint.bs23_step_vjp(f, fvjp, 0.1, g, 2e-3, yb)
    s = torch.from_numpy(g).cuda()
    ybn = torch.from_numpy(yb).cuda()
    ybar = torch.empty_like(s)
    jcb = torch.zeros_like(s)
    assert ctx.step_vjp(s, 0.1, 2e-3, ybn, ybar, jcb) == 0
    torch.cuda.synchronize()
    assert rel_l2(ybar.cpu().numpy(), ref_y) < 1e-10
    assert rel_l2(jcb.cpu().numpy(), ref_jc) < 1e-10


def test_step_fixed_matches_oracle_step():
    from oracle.bs23 import A21, A32, B1, B2, B3, C2, C3
    case = _case()
    ctx = make_gpu(case, api.FP64, fixed=3)
    ctx.set_warm_start(False)
    prob = make_oracle(case, fixed=3)
    f, _ = adjoint.film_pure_rhs(prob)
    g, t, h = case["state"], 0.1, 3e-3
    k1 = f(t, g)
    k2 = f(t + C2 * h, g + A21 * h * k1)
    k3 = f(t + C3 * h, g + A32 * h * k2)
    ref = g + h * (B1 * k1 + B2 * k2 + B3 * k3)
    s = torch.from_numpy(g.copy()).cuda()
    assert ctx.step_fixed(s, t, h) == 0
    torch.cuda.synchronize()
    assert rel_l2(s.cpu().numpy(), ref) < 1e-12


@pytest.mark.parametrize("every", [1, 2, 16])
def test_checkpointed_trajectory_gradient(every):
    """Loss <w1, y_1> + <w2, y_4> over 5 replayed steps: autograd gradients of
    g0 and the jc map equal the oracle's for every checkpoint spacing."""
    case = _case()
    ctx = make_gpu(case, api.FP64, fixed=3)
    prob = make_oracle(case, fixed=3)
    g0 = case["state"]
    steps = [2e-3, 3e-3, 1.5e-3, 2.5e-3, 2e-3]
    rng = np.random.default_rng(8)
    w1, w4 = rng.standard_normal(g0.shape), rng.standard_normal(g0.shape)
    gb_ref, jb_ref, yend = adjoint.film_trajectory_grad(prob, g0, 0.1, steps, [None, w1, None, None, w4])
    g0_t = torch.from_numpy(g0).cuda().requires_grad_(True)
    jc_t = torch.from_numpy(case["jc"]).cuda().requires_grad_(True)
    y1, y4 = ag.trajectory(ctx, g0_t, jc_t, 0.1, steps, [1, 4], every=every)
    loss = (torch.from_numpy(w1).cuda() * y1).sum() + (torch.from_numpy(w4).cuda() * y4).sum()
    loss.backward()
    assert rel_l2(y4.detach().cpu().numpy(), yend) < 1e-11
    e1 = rel_l2(g0_t.grad.cpu().numpy(), gb_ref)
    e2 = rel_l2(jc_t.grad.cpu().numpy(), jb_ref)
    print("every %d: grad rel-L2 g0 %.3e jc %.3e" % (every, e1, e2), flush=True)
    assert e1 < 1e-10 and e2 < 1e-10


def test_hz_misfit_gradient():
    """Misfit 1/2 sum (h_z - h_obs)^2 dx dy at two observed steps (the
    magneto-optical-image misfit of the gradient workload) through the
    differentiable h_z: gradient w.r.t. the jc map against the oracle."""
    case = _case()
    ctx = make_gpu(case, api.FP64, fixed=3)
    prob = make_oracle(case, fixed=3)
    g0 = case["state"]
    steps = [2e-3, 2e-3, 2e-3, 2e-3]
    rng = np.random.default_rng(12)
    obs = {1: rng.standard_normal(g0.shape) * 0.01, 3: rng.standard_normal(g0.shape) * 0.01}
    dA = prob.dx * prob.dy
    g0_t = torch.from_numpy(g0).cuda()
    jc_t = torch.from_numpy(case["jc"]).cuda().requires_grad_(True)
    ys = ag.trajectory(ctx, g0_t, jc_t, 0.1, steps, [1, 3], every=2)
    loss = 0.0
    for (k, y) in zip([1, 3], ys):
        t_k = 0.1 + sum(steps[:k + 1])
        hz = ag.hz(ctx, y, t_k)
        loss = loss + 0.5 * ((hz - torch.from_numpy(obs[k]).cuda()) ** 2).sum() * dA
    loss.backward()
    # oracle: cotangent of the state at step k is K2 (hz - obs) dA
    from oracle import film
    ys_o = []
    f, _ = adjoint.film_pure_rhs(prob)
    from oracle.bs23 import A21, A32, B1, B2, B3, C2, C3
    y, t = g0.copy(), 0.1
    bars = [None] * len(steps)
    for i, h in enumerate(steps):
        k1 = f(t, y)
        k2 = f(t + C2 * h, y + A21 * h * k1)
        k3 = f(t + C3 * h, y + A32 * h * k2)
        y, t = y + h * (B1 * k1 + B2 * k2 + B3 * k3), t + h
        if i in obs:
            hz_o, _, _ = film.observe(prob, y, t)
            bars[i] = adjoint.film_hz_vjp(prob, (hz_o - obs[i]) * dA)
    _, jb_ref, _ = adjoint.film_trajectory_grad(prob, g0, 0.1, steps, bars)
    assert rel_l2(jc_t.grad.cpu().numpy(), jb_ref) < 1e-9


@pytest.mark.parametrize("prec,tol", [(api.FP64, 1e-10), (api.MIXED, 1e-4)])
def test_checkpointed_trajectory_gradient_spectral(prec, tol):
    """The same loss and checkpointing (every 2 steps) in the spectral form of
    Sec. 2.2: gradients of g0 and the jc map against the oracle's."""
    case = _case()
    ctx = make_gpu(case, prec, fixed=3, deriv="spectral")
    prob = make_oracle(case, fixed=3, deriv="spectral")
    g0 = case["state"]
    steps = [2e-3, 3e-3, 1.5e-3, 2.5e-3, 2e-3]
    rng = np.random.default_rng(9)
    w1, w4 = rng.standard_normal(g0.shape), rng.standard_normal(g0.shape)
    gb_ref, jb_ref, yend = adjoint.film_trajectory_grad(prob, g0, 0.1, steps, [None, w1, None, None, w4])
    g0_t = torch.from_numpy(g0).cuda().requires_grad_(True)
    jc_t = torch.from_numpy(case["jc"]).cuda().requires_grad_(True)
    y1, y4 = ag.trajectory(ctx, g0_t, jc_t, 0.1, steps, [1, 4], every=2)
    loss = (torch.from_numpy(w1).cuda() * y1).sum() + (torch.from_numpy(w4).cuda() * y4).sum()
    loss.backward()
    e0 = rel_l2(y4.detach().cpu().numpy(), yend)
    e1 = rel_l2(g0_t.grad.cpu().numpy(), gb_ref)
    e2 = rel_l2(jc_t.grad.cpu().numpy(), jb_ref)
    print("spectral, precision %d: state %.3e, grad rel-L2 g0 %.3e jc %.3e" % (prec, e0, e1, e2), flush=True)
    assert e0 < tol and e1 < tol and e2 < tol
