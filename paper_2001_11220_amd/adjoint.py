"""Differentiable ETD-RDP-IF trajectories (reverse mode with checkpoints).

``trajectory(solver, u0, nsteps, params)`` returns U(T) after ``nsteps``
steps as a torch function of the initial state ``u0`` and of ``params``, the
vector (D_0..D_{s-1}, theta) the solver was built with, so that
``loss.backward()`` yields dL/du0 and dL/dparams.

Backward runs the library's one-step adjoint (``etd_rdp_adjoint``) from the
last step to the first.  The forward sweep keeps every ``checkpoint_every``-th
state; the backward sweep recomputes one segment of states at a time from its
checkpoint, so memory holds about nsteps/m + m states.  All arithmetic runs
in the library's kernels; this module only orders the calls.
"""

from __future__ import annotations

import math

import torch


class _Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, params, solver, nsteps, every):
        ctx.params_device = params.device
        u = u0.detach().clone().contiguous()
        ckpts = []
        done = 0
        while done < nsteps:
            ckpts.append(u.clone())
            n = min(every, nsteps - done)
            solver.step(u, n)
            done += n
        ctx.solver, ctx.nsteps, ctx.every, ctx.ckpts = solver, nsteps, every, ckpts
        return u

    @staticmethod
    def backward(ctx, gout):
        solver, nsteps, every = ctx.solver, ctx.nsteps, ctx.every
        lam = gout.detach().to(torch.float64).contiguous().clone()
        grad = torch.zeros(solver.grad_size, dtype=torch.float64, device=lam.device)
        if nsteps > 0:
            seg = torch.empty((min(every, nsteps),) + tuple(lam.shape), dtype=torch.float64,
                              device=lam.device)
            for i in range(len(ctx.ckpts) - 1, -1, -1):
                start = i * every
                cnt = min(every, nsteps - start)
                seg[0].copy_(ctx.ckpts[i])
                for j in range(1, cnt):
                    seg[j].copy_(seg[j - 1])
                    solver.step(seg[j], 1)
                for j in range(cnt - 1, -1, -1):
                    solver.adjoint(seg[j], lam, lam_out=lam, grad=grad)
        ctx.ckpts = None
        return lam, grad.to(device=ctx.params_device), None, None, None


def trajectory(solver, u0, nsteps, params=None, checkpoint_every=20):
    """U(T) after ``nsteps`` steps of ``solver`` (an ``etd.EtdRdp``) from
    ``u0`` (float64 device tensor of the state shape).

    ``params``: optional float64 tensor of ``solver.grad_size`` equal to
    ``solver.param_vector()``; when it requires grad, backward fills its
    gradient (D first, then the reaction parameters)."""
    if checkpoint_every < 1:
        raise ValueError("checkpoint_every must be >= 1")
    if params is None:
        params = torch.tensor(solver.param_vector(), dtype=torch.float64)
    want = solver.param_vector()
    got = [float(v) for v in params.detach().cpu().reshape(-1)]
    if len(got) != len(want) or any(not math.isclose(a, b, rel_tol=1e-15, abs_tol=0.0) for a, b in zip(got, want)):
        raise ValueError("params must equal the solver's (D, theta); build a new solver for new values")
    return _Trajectory.apply(u0, params, solver, int(nsteps), int(checkpoint_every))
