"""Differentiation form: the forward solve as a torch.autograd.Function.

``HybSolve.apply(sigma, solver, nt, dt, omega)`` returns the backscattered
trace obs[nt+1, ny+1, nx+1] (FP64) of the hybrid FEM/FDM forward sweep for
the per-cube conductivity sigma (a = 1 + sigma).  Its hand-written backward
runs the exact discrete adjoint in the HIP library (trace cotangent as the
seed, mode 1) and returns dL/dsigma (Euclidean, FP64, zero on the overlap
cubes).  With ``store_mode`` 1 or 2 on the solver, the backward restores
sqrt(nt) checkpoints and recomputes each segment of forward states in
reverse time.  No arithmetic of the method happens here.
"""
from __future__ import annotations

import torch

from . import hyb


class HybSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sigma, solver, nt, dt, omega=40.0):
        sig = sigma.detach().to(torch.float64).contiguous()
        obs = solver.forward(sig, nt, dt, omega=omega)
        ctx.solver = solver
        ctx.args = (nt, dt, omega)
        ctx.generation = solver.generation
        ctx.save_for_backward(sig)
        return obs

    @staticmethod
    def backward(ctx, grad_obs):
        solver = ctx.solver
        (sig,) = ctx.saved_tensors
        nt, dt, omega = ctx.args
        if solver.generation != ctx.generation:
            # another forward ran on this solver since: rebuild this one's states
            solver.forward(sig, nt, dt, omega=omega)
        solver.adjoint(grad_obs.to(torch.float64).contiguous(), mode=1)
        grad, _ = solver.gradient(want_J=False)
        return grad.view_as(sig), None, None, None, None


def solve(sigma, solver, nt, dt, omega=40.0):
    return HybSolve.apply(sigma, solver, nt, dt, omega)


__all__ = ["HybSolve", "solve", "hyb"]
