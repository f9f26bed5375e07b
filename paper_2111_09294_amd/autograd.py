"""torch.autograd glue: u = K^{-1} f with gradients for f and for per-element
stiffness scalings.

The forward pass is the library's solve; the backward pass is its adjoint solve
lambda = K^{-1} dL/du (K is symmetric), which is dL/df, followed by its element kernel
dL/ds_e = -lambda_e^T K_e u_e for K = sum_e s_e K_e.  Nothing is computed here.
"""
from __future__ import annotations

import torch


class _Solve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, scale, solver, elements, tol, opts):
        u, info = solver.solve(f.detach().contiguous(), tol=tol, **opts)
        ctx.solver, ctx.elements, ctx.tol, ctx.opts = solver, elements, tol, opts
        ctx.info = info
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, gu):
        (u,) = ctx.saved_tensors
        need_f, need_s = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_f or need_s):
            return None, None, None, None, None, None
        lam, _ = ctx.solver.solve_adjoint(gu.detach().contiguous(), tol=ctx.tol, **ctx.opts)
        g_s = None
        if need_s:
            if ctx.elements is None:
                raise ValueError("gradients for the element scalings need the element matrices (elements=...)")
            g_s = ctx.solver.element_gradient(ctx.elements, u, lam)
        return (lam if need_f else None), g_s, None, None, None, None


def solve(f, solver, scale=None, elements=None, tol=1e-8, **opts):
    """u = K^{-1} f by `solver`, differentiable in f and in `scale`.

    `scale` (nel, float64) stands for the per-element factors s_e of K = sum_e s_e K_e
    with which `solver` was set up: its values are not read (the caller keeps the
    solver consistent with them), it only receives dL/ds_e in the backward pass, from
    `elements` (an Elements holding the K_e).  `opts` go to Solver.solve and
    Solver.solve_adjoint (e.g. precision="mixed").
    """
    if scale is None:
        scale = torch.zeros(0, dtype=torch.float64, device=f.device)
    return _Solve.apply(f, scale, solver, elements, tol, opts)
