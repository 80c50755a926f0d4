"""Differentiable rollout: ``fv_step`` forward, ``fv_adjoint_step`` backward.

``EulerRollout.apply(U0, solver, nsteps, every)`` advances the dense interior
state ``U0`` (float64, shape (nvar, nz, ny, nx), on the solver's device) by
``nsteps`` SSP-RK3 steps and returns the final dense state. The step sizes
chosen by the CFL reduction are recorded and treated as constants (the max
reduction is not differentiable), so the gradient is that of the discrete
map at the recorded dt sequence.

Backward: checkpoints of the ghosted state are kept every ``every`` steps.
Each segment is recomputed from its checkpoint with the recorded dt, its step
states are held, and ``fv_adjoint_step`` is applied from the last step of the
segment back to its first. Device memory: nsteps / every checkpoints plus
``every`` states of one segment.
"""
from __future__ import annotations

import torch

from . import fv


class EulerRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver, nsteps, every=10, dt_in=None):
        if U0.dtype != torch.float64 or tuple(U0.shape) != tuple(solver.spec.shape):
            raise ValueError("U0 must be float64 with shape (nvar, nz, ny, nx)")
        solver.interior().copy_(U0)
        dts = torch.zeros(max(nsteps, 1), dtype=torch.float64, device=solver.device)
        if dt_in is not None:
            dts[:nsteps].copy_(dt_in[:nsteps])
        ckpts = []
        s = 0
        while s < nsteps:
            ckpts.append(solver.U.clone())
            m = min(every, nsteps - s)
            solver.step(m, dt_in=dts[s:s + m] if dt_in is not None else None, dt_out=dts[s:s + m])
            s += m
        ctx.solver = solver
        ctx.nsteps = nsteps
        ctx.every = every
        ctx.ckpts = ckpts
        ctx.dts = dts
        dts_out = dts[:nsteps].clone()
        ctx.mark_non_differentiable(dts_out)
        return solver.interior().clone(), dts_out

    @staticmethod
    def backward(ctx, gout, _gdt):
        solver = ctx.solver
        lam = gout.contiguous().clone()
        dts = ctx.dts
        nseg = len(ctx.ckpts)
        for seg in reversed(range(nseg)):
            s0 = seg * ctx.every
            m = min(ctx.every, ctx.nsteps - s0)
            solver.U.copy_(ctx.ckpts[seg])
            states = []
            for q in range(m):
                states.append(solver.U.clone())
                solver.step(1, dt_in=dts[s0 + q:s0 + q + 1])
            for q in reversed(range(m)):
                fv.fv_adjoint_step(solver.ctx, states[q].data_ptr(), dts[s0 + q:s0 + q + 1].data_ptr(),
                                   lam.data_ptr())
        ctx.ckpts = None
        return lam, None, None, None, None


def rollout(U0, solver, nsteps, every=10, dt_in=None):
    """Final state and the dt sequence used; differentiable in U0."""
    return EulerRollout.apply(U0, solver, nsteps, every, dt_in)


def pressure_integral(U, spec, window):
    """sum over cells [a, b)^2 of p * dx * dy (2D), the adjoint workload's objective."""
    a, b = window
    g1 = spec.gamma - 1.0
    rho = U[0, 0, a:b, a:b]
    mx = U[1, 0, a:b, a:b]
    my = U[2, 0, a:b, a:b]
    E = U[3, 0, a:b, a:b]
    p = g1 * (E - 0.5 * (mx * mx + my * my) / rho)
    return p.sum() * spec.dx[0] * spec.dx[1]
