"""Forward dynamics as a torch.autograd.Function whose backward is the dFD VJP.

Two modes, the same values:
  "jacobians" (default): forward runs the fused kernel (grid_fd_grad) and keeps M^-1,
      dqdd/dq and dqdd/dqd (3 n^2 floats per knot); backward runs grid_fd_vjp:
      qbar = (dqdd/dq)^T g, qdbar = (dqdd/dqd)^T g, taubar = M^-1 g.
  "adjoint": forward runs grid_fd (qdd only) and keeps q, qd, qdd; backward runs
      grid_fd_vjp_adjoint, which forms taubar = M^-1 g and the transposed products by one
      reverse sweep over RNEA (no n^2 Jacobians in memory).
Both run in the HIP library on torch's current stream; torch provides the memory.
"""
from __future__ import annotations

import torch

from . import grid


class ForwardDynamics(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, qd, tau, model, mode="jacobians"):
        q, qd, tau = (x.contiguous().float() for x in (q, qd, tau))
        ctx.model = model
        ctx.mode = mode
        stream = torch.cuda.current_stream(q.device)
        if mode == "jacobians":
            out = grid.fd_grad_torch(model, q, qd, tau)
            ctx.save_for_backward(out["Minv"], out["dqdd_dq"], out["dqdd_dqd"])
            return out["qdd"]
        if mode != "adjoint":
            raise ValueError(f"mode must be 'jacobians' or 'adjoint', not {mode!r}")
        qdd = torch.empty_like(q)
        model.fd(q, qd, tau, qdd, N=q.shape[0], stream=stream)
        ctx.save_for_backward(q, qd, qdd)
        return qdd

    @staticmethod
    def backward(ctx, g):
        g = g.contiguous().float()
        qbar = torch.empty_like(g)
        qdbar = torch.empty_like(g)
        taubar = torch.empty_like(g)
        stream = torch.cuda.current_stream(g.device)
        if ctx.mode == "jacobians":
            Minv, dq, dqd = ctx.saved_tensors
            grid.fd_vjp(ctx.model, dq, dqd, Minv, g, qbar, qdbar, taubar, N=g.shape[0],
                        stream=stream)
        else:
            q, qd, qdd = ctx.saved_tensors
            grid.fd_vjp_adjoint(ctx.model, q, qd, qdd, g, qbar, qdbar, taubar, N=g.shape[0],
                                stream=stream)
        return qbar, qdbar, taubar, None, None


def forward_dynamics(model: "grid.Model", q, qd, tau, mode: str = "jacobians"):
    """qdd = FD(q, qd, tau) for [N, n] float32 CUDA tensors, differentiable in all three."""
    return ForwardDynamics.apply(q, qd, tau, model, mode)
