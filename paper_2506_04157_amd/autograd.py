"""Differentiable Stokes solve: forward = stk_solve, backward = adjoint solve
(stk_solve_adjoint) plus the gradient kernel (stk_gradient)."""
import torch


class StokesSolve(torch.autograd.Function):
    """(u, p) = solve(K(exp(m)) [u; p] = [scale * buoyancy(T); 0]).

    m: nodal log-viscosity (P1, float64, device); T: nodal temperature (P2).
    The viscosity field is set on the context by this call.  If the
    context's fields change between this forward and its backward (another
    solve or set_* call on the same context), the backward sets the fields
    of this forward again before the adjoint solve.
    """

    @staticmethod
    def forward(ctx, m, T, sctx, params, lnrho=None, scale=1.0):
        m = m.detach().contiguous()
        lnrho = None if lnrho is None else lnrho.detach().contiguous()
        sctx.set_log_viscosity(m, lnrho, params)
        f = sctx.rhs_buoyancy(T.detach().contiguous(), scale)
        u, p, rep = sctx.solve(f, params=params)
        ctx.sctx, ctx.params, ctx.scale = sctx, params, scale
        ctx.report = rep
        ctx.generation = sctx.generation
        ctx.fields = (m, lnrho)
        ctx.save_for_backward(u)
        return u, p

    @staticmethod
    def backward(ctx, gu, gp):
        (u,) = ctx.saved_tensors
        sctx = ctx.sctx
        if sctx.generation != ctx.generation:
            m, lnrho = ctx.fields
            sctx.set_log_viscosity(m, lnrho, ctx.params)
        gu = torch.zeros_like(u) if gu is None else gu.contiguous()
        gp = sctx.zeros_p() if gp is None else gp.contiguous()
        lu, lp, _ = sctx.solve_adjoint(gu, gp, ctx.params)
        gm, gT = sctx.gradient(u, lu, ctx.scale)
        return gm, gT, None, None, None, None
