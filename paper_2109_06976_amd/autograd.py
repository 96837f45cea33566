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


class CapturedStep:
    """One forward + backward of L = sum(qdd^2) through ForwardDynamics captured in a HIP
    graph (torch.cuda.CUDAGraph), for loops that repeat the same step on new inputs.

    The inputs live in static tensors `q`, `qd`, `tau` (copy new values into them); replay()
    reruns the captured kernels, after which `loss`, `qdd` and `grads` (dL/dq, dL/dqd,
    dL/dtau) hold the results. Capture warms up on a side stream first, as torch requires.
    Every kernel of the step is an asynchronous launch on the capturing stream; the library
    calls allocate nothing and do not synchronize, so they can be captured."""

    def __init__(self, model, q, qd, tau, mode: str = "jacobians", warmup: int = 3):
        import torch as _torch
        self.model, self.mode = model, mode
        self.q, self.qd, self.tau = (x.detach().clone().contiguous().float().requires_grad_(True)
                                     for x in (q, qd, tau))
        side = _torch.cuda.Stream(device=self.q.device)
        side.wait_stream(_torch.cuda.current_stream(self.q.device))
        with _torch.cuda.stream(side):
            for _ in range(warmup):
                self._step()
        _torch.cuda.current_stream(self.q.device).wait_stream(side)
        self.graph = _torch.cuda.CUDAGraph()
        with _torch.cuda.graph(self.graph):
            self.qdd, self.loss, self.grads = self._step()

    def _step(self):
        qdd = forward_dynamics(self.model, self.q, self.qd, self.tau, self.mode)
        loss = (qdd * qdd).sum()
        grads = torch.autograd.grad(loss, (self.q, self.qd, self.tau))
        return qdd, loss, grads

    def replay(self):
        self.graph.replay()
