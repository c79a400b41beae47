"""The library's discrete adjoint behind torch.autograd.

ElderQoI.apply(xi, problem, box, dt, n_steps, checkpoint_every) returns, per sample, the
salt mass in `box` after n_steps time steps of length dt from the problem's current
states, with the porosity/permeability parameters xi [S_total, n_xi]; its backward
multiplies the incoming gradient by dJ/dxi from edf_adjoint (one backward sweep with
transposed-Jacobian multigrid solves over the trajectory that edf_solve recorded with a
checkpoint every `checkpoint_every` steps).  Both values are computed in forward.
edf_set_parameters clears the samples' sub-step history and the problem's states are
restored (edf_set_state) after the call, so J is a function of xi alone for a fixed
starting state.  Marshalling only: the time stepping and the adjoint run in the
library's kernels.
"""
import numpy as np
import torch


class ElderQoI(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xi, problem, box, dt, n_steps, checkpoint_every=10):
        x = xi.detach().to("cpu", torch.float64).numpy()
        saved = [problem.get_state(s) for s in range(problem.S)]
        try:
            problem.set_parameters(x)
            J, dJ = problem.gradient(box, dt, n_steps, checkpoint_every)
        finally:
            for s, u in enumerate(saved):
                problem.set_state(s, u)
        ctx.save_for_backward(torch.from_numpy(np.ascontiguousarray(dJ)).to(xi.device, xi.dtype))
        return torch.from_numpy(J).to(xi.device, xi.dtype)

    @staticmethod
    def backward(ctx, grad_J):
        (dJ,) = ctx.saved_tensors
        return grad_J[:, None] * dJ, None, None, None, None, None


def salt_mass(xi, problem, box, dt, n_steps, checkpoint_every=10):
    """J(xi) [S_total] as a differentiable torch function (see ElderQoI)."""
    return ElderQoI.apply(xi, problem, box, dt, n_steps, checkpoint_every)
