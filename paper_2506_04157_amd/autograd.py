"""Differentiable Stokes solve: forward = stk_solve, backward = adjoint solve
(stk_solve_adjoint) plus the gradient kernel (stk_gradient)."""
import torch


class StokesSolve(torch.autograd.Function):
    """(u, p) = solve(K(exp(m)) [u; p] = [scale * buoyancy(T); 0]).

    m: nodal log-viscosity (P1, float64, device); T: nodal temperature (P2).
    The viscosity field is set on the context by this call.
    """

    @staticmethod
    def forward(ctx, m, T, sctx, params, lnrho=None, scale=1.0):
        sctx.set_log_viscosity(m.contiguous(), lnrho, params)
        f = sctx.rhs_buoyancy(T.contiguous(), scale)
        u, p, rep = sctx.solve(f, params=params)
        ctx.sctx, ctx.params, ctx.scale = sctx, params, scale
        ctx.report = rep
        ctx.save_for_backward(u)
        return u, p

    @staticmethod
    def backward(ctx, gu, gp):
        (u,) = ctx.saved_tensors
        sctx = ctx.sctx
        gu = torch.zeros_like(u) if gu is None else gu.contiguous()
        gp = sctx.zeros_p() if gp is None else gp.contiguous()
        lu, lp, _ = sctx.solve_adjoint(gu, gp, ctx.params)
        gm, gT = sctx.gradient(u, lu, ctx.scale)
        return gm, gT, None, None, None, None
