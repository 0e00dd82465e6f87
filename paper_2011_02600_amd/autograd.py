"""torch.autograd interface of the solver: receiver traces as a
differentiable function of the nodal material (rho, lambda, mu).

The forward pass steps the solver keeping checkpoints
(sbp_step_checkpointed, receivers recorded); the backward pass runs the
library's discrete adjoint from those checkpoints
(sbp_gradient_from_checkpoints) with the incoming gradient of the traces as
the residual when the solver's checkpoints are still those of this forward
run (same checkpoint id), or else sbp_gradient from the saved initial
state.  Argument marshalling only: all
arithmetic of both passes runs in the HIP library.
"""
import numpy as np
import torch


def _cp_cs(rho, lam, mu):
    r = rho.detach().double().cpu().numpy()
    la = lam.detach().double().cpu().numpy()
    m = mu.detach().double().cpu().numpy()
    return r, np.sqrt((la + 2 * m) / r), np.sqrt(m / r)


class Seismograms(torch.autograd.Function):
    """traces = Seismograms.apply(rho, lam, mu, solver, Q0, receivers,
    nsteps, dt, every): v at the receivers after each of nsteps steps from the
    state Q0 at t = 0, shape (nsteps, nrec, 3).  Gradients flow to rho, lam
    and mu (grid functions of the solver's shape)."""

    @staticmethod
    def forward(ctx, rho, lam, mu, solver, Q0, receivers, nsteps, dt, every=100):
        solver.set_material(*_cp_cs(rho, lam, mu))
        solver.set_state(Q0, 0.0)
        traces = solver.record(receivers, nsteps)
        solver.step_checkpointed(nsteps, dt, every)
        ctx.ck_id = solver.checkpoint_id()
        ctx.solver, ctx.Q0, ctx.receivers = solver, Q0, receivers
        ctx.nsteps, ctx.dt, ctx.every = nsteps, dt, every
        ctx.mat = (rho, lam, mu)
        return traces.clone()

    @staticmethod
    def backward(ctx, grad_traces):
        s = ctx.solver
        if s.checkpoint_id() == ctx.ck_id:
            # the solver still holds this forward run's checkpoints
            g = s.gradient_from_checkpoints(grad_traces)
        else:
            # another run (e.g. a second forward pass) replaced them
            s.set_material(*_cp_cs(*ctx.mat))
            s.set_state(ctx.Q0, 0.0)
            s.record(ctx.receivers, ctx.nsteps)
            g = s.gradient(ctx.nsteps, ctx.dt, grad_traces, ctx.every)
        dev = ctx.mat[0].device
        out = [g[i].to(device=dev, dtype=ctx.mat[i].dtype) for i in range(3)]
        return out[0], out[1], out[2], None, None, None, None, None, None
