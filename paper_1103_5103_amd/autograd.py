"""torch.autograd wrapper of the Wilson-Dirac solve.

x = M(kappa; U)^{-1} b. The backward pass solves the adjoint system M^dag lam = grad_x through
M^dag = gamma5 M gamma5 (one more library solve), returns grad_b = lam, and forms the link
derivative dL/dRe U + i dL/dIm U from hopping-term outer products of x and lam in the library's
gradient kernel. The forward solution is kept for the backward pass instead of being recomputed.

The gauge handle (packed links and solver workspaces) lives as long as the autograd graph that
holds it, so a second backward (retain_graph=True) works; a caller that solves repeatedly on one
gauge field can pass its own handle and skip the packing and link checks of every call.
"""
from __future__ import annotations

import torch

from . import _lib


class WilsonSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, b, kappa, params, antiperiodic, project_su3, gauge):
        g = gauge if gauge is not None else _lib.wd_gauge_create(U.detach(), antiperiodic=antiperiodic, hint=params)
        x, st = _lib.bicgstab_solve(g, kappa, b.detach().contiguous(), p=params)
        ctx.g, ctx.kappa, ctx.params, ctx.project = g, kappa, params, project_su3
        ctx.save_for_backward(x)
        ctx.stats = st
        return x

    @staticmethod
    def backward(ctx, grad_x):
        (x,) = ctx.saved_tensors
        if not ctx.g.handle:
            raise RuntimeError("the gauge handle passed to wilson_solve was closed before the backward pass")
        p = _lib.SolverParams.from_buffer_copy(ctx.params)
        p.dagger, p.use_x0 = 1, 0
        lam, _ = _lib.bicgstab_solve(ctx.g, ctx.kappa, grad_x.contiguous(), p=p)
        gU = _lib.wd_gauge_grad(ctx.g, x, lam, project=ctx.project)
        return gU, lam, None, None, None, None, None


def wilson_solve(U, b, kappa, params=None, antiperiodic=True, project_su3=False, gauge=None):
    """x = M(kappa; U)^{-1} b with gradients for U and b. With project_su3 the gradient returned
    for U is the su(3) force F = (i/2) TA(U G^dag) instead of the complex derivative G. gauge: an
    existing handle built from the same U (its links are used; U still receives the gradient)."""
    p = _lib.params() if params is None else params
    if gauge is not None and (tuple(gauge.link_shape) != tuple(U.shape) or gauge.antiperiodic != bool(antiperiodic)):
        raise ValueError("gauge handle does not match U / antiperiodic")
    return WilsonSolve.apply(U, b, float(kappa), p, bool(antiperiodic), bool(project_su3), gauge)
