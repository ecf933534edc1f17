"""Differentiable film trajectories on the GPU (torch.autograd).

`trajectory(ctx, g0, jc_map, t0, steps, obs_steps, every)` replays the given
Bogacki-Shampine steps (mag_step_fixed, step sizes frozen) from g0 and returns
the states after the listed steps; gradients with respect to g0 and the
per-cell jc map flow back through mag_step_vjp.  Only every `every`-th state
is kept; the reverse pass recomputes one segment at a time from its
checkpoint.  Every right-hand side inside starts from dh_e/dt (the warm start
is switched off), so a step is a function of (state, t) alone and the
recomputed states are bit-identical to the forward ones.

`hz(ctx, g, t)` is the differentiable observation h_z of mag_observe.

All arithmetic runs in the HIP library; this module only orders the calls and
adds the cotangents that the loss supplies at observed steps.
"""
import torch

from . import api


class _Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(fctx, g0, jc_map, mctx, t0, steps, obs_steps, every):
        mctx.set_warm_start(False)
        mctx.set_params(jc_map, *mctx.params[1:])
        y = g0.detach().clone()
        ts = [float(t0)]
        ckpt = {0: y.clone()}
        obs = set(obs_steps)
        outs = []
        for i, h in enumerate(steps):
            st = mctx.step_fixed(y, ts[-1], h)
            if st != api.OK:
                raise api.MagError(st, "inner iteration failed during the replayed trajectory")
            ts.append(ts[-1] + h)
            if (i + 1) % every == 0:
                ckpt[i + 1] = y.clone()
            if i in obs:
                outs.append(y.clone())
        fctx.mctx, fctx.steps, fctx.ts, fctx.ckpt, fctx.every = mctx, list(steps), ts, ckpt, every
        fctx.obs_steps = list(obs_steps)
        fctx.jc_map = jc_map
        return tuple(outs)

    @staticmethod
    def backward(fctx, *grads):
        mctx, steps, ts, ckpt, every = fctx.mctx, fctx.steps, fctx.ts, fctx.ckpt, fctx.every
        mctx.set_params(fctx.jc_map, *mctx.params[1:])
        gstep = {}
        for s, g in zip(fctx.obs_steps, grads):
            if g is not None:
                gstep[s] = g.contiguous() if s not in gstep else gstep[s] + g
        ybar = torch.zeros_like(ckpt[0])
        ybar_new = torch.empty_like(ybar)
        jc_bar = torch.zeros_like(ckpt[0]) if fctx.jc_map is not None else None
        nsteps = len(steps)
        starts = list(range(0, nsteps, every))
        for s0 in reversed(starts):
            s1 = min(s0 + every, nsteps)
            y = ckpt[s0].clone()
            states = [y.clone()]
            for i in range(s0, s1 - 1):
                st = mctx.step_fixed(y, ts[i], steps[i])
                if st != api.OK:
                    raise api.MagError(st, "inner iteration failed while recomputing a segment")
                states.append(y.clone())
            for i in range(s1 - 1, s0 - 1, -1):
                if i in gstep:
                    ybar += gstep[i]
                ybar_new.copy_(ybar)
                st = mctx.step_vjp(states[i - s0], ts[i], steps[i], ybar_new, ybar, jc_bar)
                if st != api.OK:
                    raise api.MagError(st, "transposed iteration failed")
        return ybar, jc_bar, None, None, None, None, None


def trajectory(mctx, g0, jc_map, t0, steps, obs_steps, every=16):
    """States after the steps listed in obs_steps (indices into steps) of the
    replayed trajectory; differentiable with respect to g0 and jc_map (a
    float64 device tensor of cell shape, or None for the uniform jc0)."""
    if jc_map is None:
        jc_map_t = None
    else:
        jc_map_t = jc_map
    return _Trajectory.apply(g0, jc_map_t, mctx, float(t0), list(steps), list(obs_steps), int(every))


class _Hz(torch.autograd.Function):
    @staticmethod
    def forward(fctx, g, mctx, t):
        fctx.mctx = mctx
        hz, _, _ = mctx.observe(g.detach().contiguous(), t, want_hz=True, want_j=False)
        return hz

    @staticmethod
    def backward(fctx, hz_bar):
        gbar = torch.empty_like(hz_bar)
        fctx.mctx.observe_vjp(hz_bar.contiguous(), gbar)
        return gbar, None, None


def hz(mctx, g, t):
    """h_z = h_e + F^{-1}[|k|/2 F(g)] on the nodes (film), differentiable in g."""
    return _Hz.apply(g, mctx, float(t))
