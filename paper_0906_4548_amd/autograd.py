"""torch.autograd.Function wrappers of the solve, the CIC deposit and interpolation, and the
binned power spectrum of C.  Forward and backward both call the C-ABI; torch supplies
memory and streams only.

    delta = CICDeposit.apply(pos, plan)                 # dL/dpos via the CIC adjoint
    u     = FieldSolve.apply(delta, plan, params)       # dL/ddelta via the implicit adjoint
    f     = CICInterp.apply(mesh, pos, plan)            # dL/dmesh, dL/dpos via the CIC adjoint
    pk    = PowerOfC.apply(u, plan, params, nbins)      # [batch, nbins]
"""
import warnings

import numpy as np
import torch

from . import dgp


class SolveNotConvergedError(RuntimeError):
    """The gradient of a solve that did not converge (or of an adjoint that did not) is not the
    implicit adjoint of a solution of the field equation."""


class FieldSolve(torch.autograd.Function):
    """u* = solve(delta); backward solves J^T mu = dL/du and returns S mu (float64).

    A forward solve that stops without meeting its tolerance (DGP_NOT_CONVERGED, or
    DGP_BAD_POINTS where bad points leave vertex values at which the adjoint is undefined) warns
    in forward and raises SolveNotConvergedError in backward; so does an adjoint solve that
    reaches its max_iter."""

    @staticmethod
    def forward(ctx, delta, plan, prm, bwd_prm=None):
        u = torch.zeros_like(delta, dtype=torch.float64)
        st, info = plan.solve_field(prm, delta.contiguous(), u)
        ctx.plan, ctx.prm = plan, (bwd_prm if bwd_prm is not None else prm)
        ctx.info = info
        ctx.status = st
        if st != dgp._lib.DGP_OK:
            warnings.warn("field solve returned status %d (%s): its gradient is not defined"
                          % (st, [i["status"] for i in info]), RuntimeWarning, stacklevel=2)
        ctx.save_for_backward(delta, u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        if ctx.status != dgp._lib.DGP_OK:
            raise SolveNotConvergedError("backward through a field solve that ended with status %d" % ctx.status)
        delta, u = ctx.saved_tensors
        grad_delta = torch.zeros_like(delta)
        st, info = ctx.plan.solve_field_backward(ctx.prm, delta.contiguous(), u,
                                                 grad_u.contiguous().to(torch.float64), grad_delta)
        if st != dgp._lib.DGP_OK:
            raise SolveNotConvergedError("implicit adjoint did not converge (status %d, residuals %s)"
                                         % (st, [i["resid"] for i in info]))
        return grad_delta, None, None, None


class CICInterp(torch.autograd.Function):
    """out [ncomp, np] = CIC interpolation of mesh [ncomp, N^3] (float64) at pos [3, np];
    backward: dL/dmesh (deterministic transposed scatter) and dL/dpos (dW/dx weights)."""

    @staticmethod
    def forward(ctx, mesh, pos, plan):
        nc = mesh.numel() // plan.n3
        out = torch.zeros((nc, pos.shape[-1]), dtype=torch.float64, device=pos.device)
        plan.interp(mesh.contiguous(), pos.contiguous(), out)
        ctx.plan = plan
        ctx.save_for_backward(mesh, pos)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        mesh, pos = ctx.saved_tensors
        want_mesh, want_pos = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        grad_mesh = torch.zeros_like(mesh, dtype=torch.float64) if want_mesh else None
        grad_pos = torch.zeros(pos.shape, dtype=torch.float64, device=pos.device) if want_pos else None
        if want_mesh or want_pos:
            ctx.plan.interp_backward(mesh.contiguous(), pos.contiguous(), grad_out.contiguous().to(torch.float64),
                                     grad_pos, grad_mesh)
        return grad_mesh, (grad_pos.to(pos.dtype) if want_pos else None), None


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
