"""torch.autograd.Function over a whole fixed-dt time integration of a 2D scalar
conservation law (hybrid HWENO stage operator of Section 2.2 inside TVD-RK3, eq. RK).

Forward: the library advances U0 by nsteps steps, keeping a checkpoint every k steps.
Backward: the library replays each k-step segment from its checkpoint and runs the
hand-written stage reverses (troubled-cell flags, hybrid masks and Lax-Friedrichs speeds
held at their forward values), returning dLoss/dU0.  Only device tensors cross."""
import torch

from .solver import Solver


class HWENOSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver, nsteps, dt, k):
        solver.set_state_tensor(U0)
        solver.forward_ckpt(nsteps, dt, k)
        ctx.solver = solver
        return solver.get_state_tensor()

    @staticmethod
    def backward(ctx, grad_out):
        g = ctx.solver.adjoint(grad_out.contiguous())
        return g, None, None, None, None


def solve(U0, solver: Solver, nsteps: int, dt: float, k: int = 20):
    """U(T) for U0 (device tensor (3, 1, ny, nx), float64), differentiable in U0.  A
    solver records one run at a time: call backward before the next solve on it."""
    return HWENOSolve.apply(U0, solver, int(nsteps), float(dt), int(k))
