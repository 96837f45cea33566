"""Forward dynamics as a torch.autograd.Function whose backward is the dFD VJP.

forward(q, qd, tau) runs the fused kernel (grid_fd_grad) and keeps M^-1, dqdd/dq and
dqdd/dqd; backward(g) runs grid_fd_vjp: qbar = (dqdd/dq)^T g, qdbar = (dqdd/dqd)^T g,
taubar = M^-1 g. Both run in the HIP library on torch's current stream; torch provides
the memory.
"""
from __future__ import annotations

import torch

from . import grid


class ForwardDynamics(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, qd, tau, model):
        q, qd, tau = (x.contiguous().float() for x in (q, qd, tau))
        out = grid.fd_grad_torch(model, q, qd, tau)
        ctx.model = model
        ctx.save_for_backward(out["Minv"], out["dqdd_dq"], out["dqdd_dqd"])
        return out["qdd"]

    @staticmethod
    def backward(ctx, g):
        Minv, dq, dqd = ctx.saved_tensors
        g = g.contiguous().float()
        qbar = torch.empty_like(g)
        qdbar = torch.empty_like(g)
        taubar = torch.empty_like(g)
        grid.fd_vjp(ctx.model, dq, dqd, Minv, g, qbar, qdbar, taubar, N=g.shape[0],
                    stream=torch.cuda.current_stream(g.device))
        return qbar, qdbar, taubar, None


def forward_dynamics(model: "grid.Model", q, qd, tau):
    """qdd = FD(q, qd, tau) for [N, n] float32 CUDA tensors, differentiable in all three."""
    return ForwardDynamics.apply(q, qd, tau, model)
