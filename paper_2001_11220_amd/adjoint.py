"""Differentiable ETD-RDP-IF trajectories (reverse mode with checkpoints).

``trajectory(solver, u0, nsteps, params)`` returns U(T) after ``nsteps``
steps as a torch function of the initial state ``u0`` and of ``params``, the
vector (D_0..D_{s-1}, theta) the solver was built with, so that
``loss.backward()`` yields dL/du0 and dL/dparams.

Backward runs the library's one-step adjoint from the last step to the
first.  Two memory plans:

* stored (``keep`` true): the forward sweep keeps every state and every
  step's carried arrays (``step_keep``), and the backward sweep runs the
  reverse steps on them (``adjoint(..., kept=...)``), with no forward work
  left: about (1 + keep_bytes / state_bytes) states of memory per step;
* checkpointed (``keep`` false): the forward sweep keeps every
  ``checkpoint_every``-th state; the backward sweep recomputes one segment
  at a time from its checkpoint, keeping that segment's carried arrays, so
  memory holds about nsteps/m states plus m steps' kept arrays.

``keep="auto"`` stores when the stored plan takes at most half the free
device memory.  Both plans give the same result bit for bit (the kept
arrays are exactly what a reverse step would recompute).  All arithmetic
runs in the library's kernels; this module only orders the calls.
"""

from __future__ import annotations

import math

import torch


def _stored_fits(solver, u, nsteps):
    free, _ = torch.cuda.mem_get_info(u.device)
    need = nsteps * (solver.keep_bytes + u.numel() * u.element_size())
    return need <= 0.5 * free


class _Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, params, solver, nsteps, every, keep):
        ctx.params_device = params.device
        u = u0.detach()
        if keep == "auto":
            keep = nsteps > 0 and _stored_fits(solver, u, nsteps)
        ctx.stored = bool(keep)
        if ctx.stored:
            # states[i + 1] = step(states[i]) out of place: no copies
            states = torch.empty((nsteps + 1,) + tuple(u.shape), dtype=u.dtype, device=u.device)
            states[0].copy_(u)
            kept = solver.new_keep(nsteps)
            for i in range(nsteps):
                solver.step_keep(states[i], kept[i], out=states[i + 1])
            u = states[nsteps].clone()
            ctx.states, ctx.kept = states, kept
        else:
            u = u.clone().contiguous()
            ckpts = []
            done = 0
            while done < nsteps:
                ckpts.append(u.clone())
                n = min(every, nsteps - done)
                solver.step(u, n)
                done += n
            ctx.ckpts = ckpts
        ctx.solver, ctx.nsteps, ctx.every = solver, nsteps, every
        return u

    @staticmethod
    def backward(ctx, gout):
        solver, nsteps, every = ctx.solver, ctx.nsteps, ctx.every
        lam = gout.detach().to(torch.float64).contiguous().clone()
        grad = torch.zeros(solver.grad_size, dtype=torch.float64, device=lam.device)
        if ctx.stored:
            for i in range(nsteps - 1, -1, -1):
                solver.adjoint(ctx.states[i], lam, lam_out=lam, grad=grad, kept=ctx.kept[i])
            ctx.states = ctx.kept = None
        elif nsteps > 0:
            m = min(every, nsteps)
            # a segment's states: its checkpoint, then seg[1..cnt-1]; seg[0]
            # takes the output of its last step, which the reverse sweep
            # does not need
            seg = torch.empty((m,) + tuple(lam.shape), dtype=torch.float64, device=lam.device)
            kept = solver.new_keep(m)
            for i in range(len(ctx.ckpts) - 1, -1, -1):
                cnt = min(every, nsteps - i * every)
                st = [ctx.ckpts[i]] + [seg[j] for j in range(1, cnt)]
                for j in range(cnt):
                    solver.step_keep(st[j], kept[j], out=st[j + 1] if j + 1 < cnt else seg[0])
                for j in range(cnt - 1, -1, -1):
                    solver.adjoint(st[j], lam, lam_out=lam, grad=grad, kept=kept[j])
            ctx.ckpts = None
        return lam, grad.to(device=ctx.params_device), None, None, None, None


def trajectory(solver, u0, nsteps, params=None, checkpoint_every=20, keep="auto"):
    """U(T) after ``nsteps`` steps of ``solver`` (an ``etd.EtdRdp``) from
    ``u0`` (float64 device tensor of the state shape).

    ``params``: optional float64 tensor of ``solver.grad_size`` equal to
    ``solver.param_vector()``; when it requires grad, backward fills its
    gradient (D first, then the reaction parameters).  ``keep``: True (store
    every step's carried arrays), False (checkpoints every
    ``checkpoint_every`` steps) or "auto" (store when it fits in half the
    free device memory)."""
    if checkpoint_every < 1:
        raise ValueError("checkpoint_every must be >= 1")
    if keep not in (True, False, "auto"):
        raise ValueError('keep must be True, False or "auto"')
    if params is None:
        params = torch.tensor(solver.param_vector(), dtype=torch.float64)
    want = solver.param_vector()
    got = [float(v) for v in params.detach().cpu().reshape(-1)]
    if len(got) != len(want) or any(not math.isclose(a, b, rel_tol=1e-15, abs_tol=0.0) for a, b in zip(got, want)):
        raise ValueError("params must equal the solver's (D, theta); build a new solver for new values")
    return _Trajectory.apply(u0, params, solver, int(nsteps), int(checkpoint_every), keep)
