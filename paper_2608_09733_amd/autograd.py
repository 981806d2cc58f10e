"""torch.autograd bridge over the adjoint path.

`Energy.apply(params, circuit_ops, ham, state)` returns E(theta) = <psi(theta)|H|psi(theta)>
with psi(theta) = U(theta)|0..0>; its backward returns grad_out * dE/dtheta.
One library call (sv_adjoint_grad_device) computes E and the whole gradient
on the GPU with the adjoint method (one forward sweep, lambda = H psi, one
backward sweep); forward keeps the gradient for backward, so a training step
costs one such call and no parameter-shift evaluations.

    st = sv.State(n, adjoint=True)
    theta = torch.rand(P, dtype=torch.float64, device="cuda", requires_grad=True)
    e = Energy.apply(theta, circ.ops, ham, st)
    e.backward()            # theta.grad = dE/dtheta
"""
from __future__ import annotations

import torch

from . import sv


class Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, ops, ham, state: "sv.State", op_array=None):
        if params.dim() != 1 or params.dtype != torch.float64:
            raise ValueError("params must be a 1-D float64 tensor")
        host = params.detach().to("cpu").numpy()
        out = torch.empty(1 + host.size, dtype=torch.float64, device="cuda")
        state.reset()
        state.adjoint_grad_device(ops, host, ham, out, op_array=op_array)
        grad = out[1:].to(params.device)
        ctx.save_for_backward(grad)
        return out[0].to(params.device)

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        return grad_out * grad, None, None, None, None


def energy(params: torch.Tensor, ops, ham, state: "sv.State", op_array=None) -> torch.Tensor:
    """E(theta) as a differentiable scalar tensor."""
    return Energy.apply(params, ops, ham, state, op_array)
