"""Trajectories of the Yoshida integrator as a differentiable torch operation.

:func:`trajectory` maps an initial state (q0, p0) to the state after ``nsteps``
steps of ``dt`` (eq. 4, forces of the context's model) and is differentiable with
respect to q0 and p0.  The forward pass runs ``md_step`` in segments of
``checkpoint_every`` steps and keeps only the state at each segment start; the
backward pass walks the segments in reverse, and for each one ``md_step_vjp``
recomputes the segment from its checkpoint and sweeps the adjoints back through
it (Hessian-vector products of the potential for the kicks).  Memory: one
checkpoint per segment plus the stage buffer of one segment.  With
``checkpoint_every = 0`` the forward records every kick position instead and the
backward needs no recomputation (3 nsteps position arrays of device memory).

Gradients are those of the discrete map (the integrator as computed), not of the
exact flow.
"""
from __future__ import annotations

import torch

from . import md


class _RecordedTrajectory(torch.autograd.Function):
    """No recomputation: the forward records every kick position (md_step_record)
    and the backward sweeps over them (md_step_vjp_recorded)."""

    @staticmethod
    def forward(fctx, q0, p0, ctx, dt, nsteps):
        q = q0.detach().clone()
        p = p0.detach().clone()
        f = torch.empty_like(q)
        md.md_force(ctx, q, f)
        start = q.clone()
        stage = md.md_step_record(ctx, q, p, f, dt, nsteps)
        fctx.save_for_backward(start, stage)
        fctx.mdctx, fctx.dt, fctx.nsteps = ctx, dt, nsteps
        return q, p

    @staticmethod
    def backward(fctx, gq, gp):
        start, stage = fctx.saved_tensors
        lq = (gq.detach().clone() if gq is not None else torch.zeros_like(start)).contiguous()
        lp = (gp.detach().clone() if gp is not None else torch.zeros_like(start)).contiguous()
        md.md_step_vjp_recorded(fctx.mdctx, start, fctx.dt, fctx.nsteps, lq, lp, stage)
        return lq, lp, None, None, None


class _Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(fctx, q0, p0, ctx, dt, nsteps, checkpoint_every):
        q = q0.detach().clone()
        p = p0.detach().clone()
        f = torch.empty_like(q)
        md.md_force(ctx, q, f)
        starts = []
        segs = []
        done = 0
        while done < nsteps:
            k = min(checkpoint_every, nsteps - done)
            starts.append(q.clone())
            starts.append(p.clone())
            segs.append(k)
            md.md_step(ctx, q, p, f, dt, k)
            done += k
        fctx.save_for_backward(*starts)
        fctx.mdctx, fctx.dt, fctx.segs = ctx, dt, segs
        return q, p

    @staticmethod
    def backward(fctx, gq, gp):
        starts = fctx.saved_tensors
        ctx = fctx.mdctx
        lq = gq.detach().clone() if gq is not None else torch.zeros_like(starts[0])
        lp = gp.detach().clone() if gp is not None else torch.zeros_like(starts[1])
        lq = lq.contiguous()
        lp = lp.contiguous()
        kmax = max(fctx.segs) if fctx.segs else 0
        stage = torch.empty(max(md.md_vjp_stage_bytes(ctx, kmax), 8), dtype=torch.uint8, device=lq.device)
        for s in range(len(fctx.segs) - 1, -1, -1):
            md.md_step_vjp(ctx, starts[2 * s], starts[2 * s + 1], fctx.dt, fctx.segs[s], lq, lp, stage)
        return lq, lp, None, None, None, None


def trajectory(ctx: md.Context, q0: torch.Tensor, p0: torch.Tensor, dt: float, nsteps: int,
               checkpoint_every: int = 50):
    """(q, p) after nsteps steps from (q0, p0); differentiable in q0 and p0.

    checkpoint_every = k >= 1 keeps the state every k steps and recomputes each
    segment in the backward pass; checkpoint_every = 0 records every kick position
    instead (md_record_stage_bytes(ctx, nsteps) of device memory, no recompute)."""
    if checkpoint_every < 0:
        raise ValueError("checkpoint_every must be >= 0")
    if checkpoint_every == 0:
        return _RecordedTrajectory.apply(q0, p0, ctx, float(dt), int(nsteps))
    return _Trajectory.apply(q0, p0, ctx, float(dt), int(nsteps), int(checkpoint_every))


def kinetic_energy_gradient(ctx: md.Context, q0: torch.Tensor, p0: torch.Tensor, dt: float, nsteps: int,
                            checkpoint_every: int = 50):
    """(K_T, dK_T/dq0, dK_T/dp0) for the final kinetic energy K_T = |p_T|^2 / 2."""
    q0 = q0.detach().clone().requires_grad_(True)
    p0 = p0.detach().clone().requires_grad_(True)
    _, pT = trajectory(ctx, q0, p0, dt, nsteps, checkpoint_every)
    K = 0.5 * (pT * pT).sum()
    K.backward()
    return K.detach(), q0.grad, p0.grad


def magnetization_gradient(ctx: md.Context, q0: torch.Tensor, p0: torch.Tensor, dt: float, nsteps: int,
                           checkpoint_every: int = 50):
    """(M_T, dM_T/dq0, dM_T/dp0) for the final magnetization modulus
    M_T = |(1/N) sum_i (cos q_i, sin q_i)| of an angle model (HMF eq. 7; also the
    order parameter of the Ring model).  Only the observable is differentiated by
    torch; the trajectory's derivative is md_step_vjp."""
    if q0.shape[0] != 1:
        raise ValueError("magnetization_gradient: angle models (HMF, Ring) only")
    q0 = q0.detach().clone().requires_grad_(True)
    p0 = p0.detach().clone().requires_grad_(True)
    qT, _ = trajectory(ctx, q0, p0, dt, nsteps, checkpoint_every)
    M = torch.sqrt(torch.cos(qT).mean() ** 2 + torch.sin(qT).mean() ** 2)
    M.backward()
    return M.detach(), q0.grad, p0.grad

