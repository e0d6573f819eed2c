"""torch.autograd.Function over the solver: n explicit steps from a conserved state, with the
jet Mach number, jet density and tau_ref as differentiable parameters.  The backward pass is
the library's hand-written discrete adjoint (maxent_step_adjoint) over the recorded time
steps, with checkpointed recomputation; torch only holds device memory and streams."""
import torch

from .solver import MaxEntSolver


class MaxEntSteps(torch.autograd.Function):
    """U_n = MaxEntSteps.apply(U0, params, solver, n, dt, checkpoint_every)

    U0       conserved state [14][ny][nx], float64 CUDA tensor
    params   tensor [jet Mach, jet rho, tau_ref] (float64, any device)
    solver   a MaxEntSolver (14 moments, FP64); its state is overwritten, and it must not be
             used again before the backward pass (which raises if it was)
    n        number of steps; dt > 0 fixed, <= 0 CFL (the recorded steps are frozen in the
             backward pass)
    """

    @staticmethod
    def forward(ctx, U0, params, solver, n, dt=0.0, checkpoint_every=20):
        if not isinstance(solver, MaxEntSolver):
            raise TypeError('solver must be a MaxEntSolver')
        p = params.detach().to('cpu', torch.float64)
        solver.record(0, 1)
        solver.set_inflow(float(p[0]), float(p[1]))
        solver.init_state(U0.detach(), repr='conserved')
        solver.record(checkpoint_every, max(int(n), 1))
        solver.step(int(n), dt=float(dt), tau_ref=float(p[2]))
        ctx.solver = solver
        ctx.generation = solver.generation
        ctx.params_device = params.device
        return solver.get('conserved')

    @staticmethod
    def backward(ctx, gU):
        if ctx.solver.generation != ctx.generation:
            raise RuntimeError('the solver was used (init_state, record, step or set_inflow) after '
                               'this forward pass: its tape no longer holds these steps')
        gU0, g = ctx.solver.adjoint(gU.contiguous(), want_dU0=True)
        gp = torch.tensor(g, dtype=torch.float64, device=ctx.params_device)
        return gU0, gp, None, None, None, None
