"""torch.autograd view of the adjoint: J(eps_r) with dJ/d eps_r from sbp_adjoint.

``PermittivityObjective(problem, block, nsteps, region)`` wraps one context.
Calling it with a tensor of per-cell eps_r for ``block`` (shape (nz, ny, nx))
sets the block's permittivity, runs the problem for ``nsteps`` steps from the
state it had when the objective was created, and returns

    J = dt * sum_{n=1..N} sum_{cells in region} |Ebar^n|^2

as a 0-d tensor.  When autograd will need the gradient, the forward call
runs the reverse sweep on the GPU as well (sbp_adjoint computes J and the
gradient together) and ``backward`` only scales the stored gradient;
otherwise it runs the forward steps alone.  All arithmetic runs in the HIP
library.
"""
import numpy as np
import torch

from .binding import build_problem


class _EpsObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps_r, obj):
        grad = obj._evaluate(eps_r, with_grad=ctx.needs_input_grad[0])
        if grad is not None:
            ctx.save_for_backward(grad)
        return torch.tensor(obj.last_J, dtype=torch.float64, device=eps_r.device)

    @staticmethod
    def backward(ctx, gJ):
        (grad,) = ctx.saved_tensors
        return gJ * grad, None


class PermittivityObjective:
    """Region objective of one block as a differentiable function of its
    per-cell relative permittivity."""

    def __init__(self, problem, block, nsteps, region, ckpt_every=0, prec=None, stream=None, history=None):
        self.problem = problem
        self.block = int(block)
        self.nsteps = int(nsteps)
        self.region = tuple(int(v) for v in region)
        self.ckpt_every = int(ckpt_every)
        self.ctx = build_problem(problem, prec=prec, stream=stream,
                                 history=history or max(self.nsteps + 8, 64))
        nbytes = self.ctx.state_bytes()
        self._start = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self._nbytes = nbytes
        self.ctx.save_state(self._start.data_ptr(), nbytes)
        blk = problem["blocks"][self.block]
        self._mu = blk.get("mu_r")
        self._sigma = blk.get("sigma")
        self.shape = (blk["n"][2], blk["n"][1], blk["n"][0])
        self.last_J = None

    def _evaluate(self, eps_r, with_grad=True):
        if tuple(eps_r.shape) != self.shape:
            raise ValueError(f"eps_r must have shape {self.shape}")
        e = eps_r.detach().to("cpu", torch.float64).numpy()
        self.ctx.set_materials(self.block, np.ascontiguousarray(e), self._mu, self._sigma)
        self.ctx.load_state(self._start.data_ptr(), self._nbytes)
        if not with_grad:  # J alone: the forward steps, no reverse sweep
            self.last_J = self.ctx.adjoint(self.block, self.nsteps, self.region, None, self.ckpt_every)
            return None
        grad = torch.zeros(self.shape, dtype=torch.float64, device="cuda")
        self.last_J = self.ctx.adjoint(self.block, self.nsteps, self.region, grad.data_ptr(), self.ckpt_every)
        return grad.to(eps_r.device)

    def __call__(self, eps_r):
        return _EpsObjective.apply(eps_r, self)

    def close(self):
        self.ctx.close()
