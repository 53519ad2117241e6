"""torch.autograd binding of the reverse-mode entry points of librrt.

RRTFunction.apply(w, n_H, solver, K) -> (lnGamma, x): K unrolled
order-independent iterations from the optically thin state, with the bin
weights w (length n_bins) and the particle densities n_H (length n) as
differentiable inputs.  The backward pass runs rrt_backward on the GPU.

The solver keeps the iterates of its most recent forward only.  Each forward
carries the solver's forward count; a backward whose forward is no longer the
solver's most recent raises instead of returning the gradient at other
parameters.
"""
from __future__ import annotations

import torch


class RRTFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w, n_H, solver, K):
        solver.set_spectrum(solver.sigma, w.detach().to(torch.float64).cpu().numpy())
        solver.set_density(n_H.detach())
        lnG, x = solver.forward(int(K))
        ctx.solver = solver
        ctx.generation = solver.generation
        ctx.w_meta = (w.dtype, w.device)
        ctx.n_meta = (n_H.dtype, n_H.device)
        return lnG, x

    @staticmethod
    def backward(ctx, g_lnG, g_x):
        if ctx.solver.generation != ctx.generation:
            raise RuntimeError("RRTFunction.backward: the solver ran another forward since this "
                               "one; its iterates are gone (use one solver per graph)")
        dw, dn = ctx.solver.backward(g_lnG, g_x)
        dw = torch.from_numpy(dw).to(dtype=ctx.w_meta[0], device=ctx.w_meta[1])
        dn = dn.to(dtype=ctx.n_meta[0], device=ctx.n_meta[1])
        return dw, dn, None, None


def log10_rate_loss(lnG: torch.Tensor, lnG_target: torch.Tensor) -> torch.Tensor:
    """sum_p (log10 Gamma_p - log10 Gamma_target,p)^2 from natural-log rates."""
    ln10 = 2.302585092994046
    return torch.sum(((lnG - lnG_target) / ln10) ** 2)
