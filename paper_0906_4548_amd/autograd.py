"""torch.autograd.Function wrappers of the solve, the CIC deposit and the binned
power spectrum of C.  Forward and backward both call the C-ABI; torch supplies
memory and streams only.

    delta = CICDeposit.apply(pos, plan)                 # dL/dpos via the CIC adjoint
    u     = FieldSolve.apply(delta, plan, params)       # dL/ddelta via the implicit adjoint
    pk    = PowerOfC.apply(u, plan, params, nbins)      # [batch, nbins]
"""
import numpy as np
import torch

from . import dgp


class FieldSolve(torch.autograd.Function):
    """u* = solve(delta); backward solves J^T mu = dL/du and returns S mu (float64)."""

    @staticmethod
    def forward(ctx, delta, plan, prm, bwd_prm=None):
        u = torch.zeros_like(delta, dtype=torch.float64)
        st, info = plan.solve_field(prm, delta.contiguous(), u)
        ctx.plan, ctx.prm = plan, (bwd_prm if bwd_prm is not None else prm)
        ctx.info = info
        ctx.save_for_backward(delta, u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        delta, u = ctx.saved_tensors
        grad_delta = torch.zeros_like(delta)
        ctx.plan.solve_field_backward(ctx.prm, delta.contiguous(), u, grad_u.contiguous().to(torch.float64),
                                      grad_delta)
        return grad_delta, None, None, None


class CICDeposit(torch.autograd.Function):
    """delta (float64 [N^3]) from positions [3, np]; backward: (N^3/np) sum_c g_c dW_c/dx."""

    @staticmethod
    def forward(ctx, pos, plan):
        delta = torch.zeros(plan.n3, dtype=torch.float64, device=pos.device)
        plan.deposit(pos.contiguous(), None, delta)
        ctx.plan = plan
        ctx.save_for_backward(pos)
        return delta

    @staticmethod
    def backward(ctx, grad_delta):
        (pos,) = ctx.saved_tensors
        grad_pos = torch.zeros(pos.shape, dtype=torch.float64, device=pos.device)
        ctx.plan.deposit_backward(pos.contiguous(), grad_delta.contiguous().to(torch.float64), grad_pos)
        return grad_pos.to(pos.dtype), None


class PowerOfC(torch.autograd.Function):
    """Binned P(k) of C = lapbar^{-1} u for each batch element: [batch, nbins] float64 (on u's device)."""

    @staticmethod
    def forward(ctx, u, plan, prm, nbins=64):
        pk, cnt = plan.power_spectrum(prm, u.contiguous(), of_c=True, nbins=nbins)
        ctx.plan, ctx.prm, ctx.nbins = plan, prm, nbins
        ctx.save_for_backward(u)
        return torch.from_numpy(pk).to(u.device)

    @staticmethod
    def backward(ctx, grad_pk):
        (u,) = ctx.saved_tensors
        grad_u = torch.zeros_like(u)
        g = np.ascontiguousarray(grad_pk.detach().to("cpu", torch.float64).numpy())
        ctx.plan.power_spectrum_backward(ctx.prm, u.contiguous(), g, grad_u, of_c=True)
        return grad_u, None, None, None


def power_loss(pk, target, weights):
    """sum_b w_b (P_b - T_b)^2 (the differentiation config's loss; plain torch on 64 numbers)."""
    return torch.sum(weights * (pk - target) ** 2)
