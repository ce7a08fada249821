"""torch.autograd wrappers of the libhb entry points.  Argument marshalling
and autograd plumbing only: the residual, the forces, the steady-state
iteration and every reverse-mode product run in the HIP library.

  residual(grid, q, xy=None, alpha0=None)   R*(q; X, alpha0)      hb_residual
  forces(grid, q, xy=None, alpha0=None)     cf(q; X, alpha0)      hb_forces
  steady_state(grid, q0, xy, alpha0, n_iter, n_adj_iter)
                                            q* with R*(q*) = 0    hb_rk_iterate

Backward passes: hb_residual_adjoint, hb_forces_adjoint and, for the steady
state, the implicit-function adjoint: with qbar* the incoming gradient,
lambda solves J_Q^T lambda = -qbar* (hb_adjoint_iterate) and the gradients
of X and alpha0 are lambda^T dR*/dX and lambda^T dR*/d alpha0
(hb_residual_adjoint).  The steady state does not depend on its starting
point, so q0 receives no gradient.

X (node coordinates, hb_xy_size() doubles, device) and alpha0 (a 0-dim
float64 tensor on any device, or a Python float) are set on the grid before
each forward and again before each backward evaluation, so the grid's
geometry after a call is that of the last evaluation.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import hb


def _set_geometry(grid: "hb.Grid", xy, alpha0):
    if xy is not None:
        grid.set_xy(xy.detach().contiguous())
    if alpha0 is not None:
        grid.set_alpha0(float(alpha0))


def _alpha_grad(ab, alpha0):
    if ab is None or not isinstance(alpha0, torch.Tensor):
        return None
    return ab.reshape(alpha0.shape).to(alpha0.device)


def _bars(grid, ctx, i_xy, i_alpha, dev):
    xyb = torch.empty(grid.n_xy, dtype=torch.float64, device=dev) \
        if ctx.needs_input_grad[i_xy] else None
    ab = torch.empty(1, dtype=torch.float64, device=dev) if ctx.needs_input_grad[i_alpha] else None
    return xyb, ab


class ResidualFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, grid, q, xy, alpha0):
        _set_geometry(grid, xy, alpha0)
        ctx.grid, ctx.alpha0 = grid, alpha0
        ctx.save_for_backward(q, xy)
        return grid.residual(q.detach().contiguous())

    @staticmethod
    def backward(ctx, rbar):
        q, xy = ctx.saved_tensors
        g = ctx.grid
        _set_geometry(g, xy, ctx.alpha0)
        xyb, ab = _bars(g, ctx, 2, 3, q.device)
        qb = g.residual_adjoint(q.detach(), rbar.contiguous(), None, xyb, ab)
        return None, qb if ctx.needs_input_grad[1] else None, xyb, _alpha_grad(ab, ctx.alpha0)


class ForceFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, grid, q, xy, alpha0):
        _set_geometry(grid, xy, alpha0)
        ctx.grid, ctx.alpha0 = grid, alpha0
        ctx.save_for_backward(q, xy)
        return grid.forces(q.detach().contiguous())

    @staticmethod
    def backward(ctx, cfbar):
        q, xy = ctx.saved_tensors
        g = ctx.grid
        _set_geometry(g, xy, ctx.alpha0)
        xyb, ab = _bars(g, ctx, 2, 3, q.device)
        qb = g.forces_adjoint(q.detach(), cfbar.contiguous(), None, xyb, ab)
        return None, qb if ctx.needs_input_grad[1] else None, xyb, _alpha_grad(ab, ctx.alpha0)


class SteadyStateFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, grid, q0, xy, alpha0, n_iter, n_adj_iter):
        _set_geometry(grid, xy, alpha0)
        q = q0.detach().clone().contiguous()
        norms = torch.empty(max(1, n_iter), dtype=torch.float64, device=q.device)
        if n_iter > 0:
            grid.rk_iterate(q, n_iter, norms[:n_iter])
        ctx.grid, ctx.alpha0, ctx.n_adj = grid, alpha0, n_adj_iter
        ctx.save_for_backward(q, xy)
        grid.last_norms = norms[:n_iter]
        return q

    @staticmethod
    def backward(ctx, qbar):
        q, xy = ctx.saved_tensors
        g = ctx.grid
        _set_geometry(g, xy, ctx.alpha0)
        lam = torch.zeros_like(q)
        norms = torch.empty(max(1, ctx.n_adj), dtype=torch.float64, device=q.device)
        if ctx.n_adj > 0:
            g.adjoint_iterate(q, lam, qbar.contiguous(), ctx.n_adj, norms[:ctx.n_adj])
        g.last_adjoint_norms = norms[:ctx.n_adj]
        g.last_lambda = lam
        xyb, ab = _bars(g, ctx, 2, 3, q.device)
        if xyb is not None or ab is not None:
            g.residual_adjoint(q, lam, None, xyb, ab)
        return None, None, xyb, _alpha_grad(ab, ctx.alpha0), None, None


def residual(grid, q, xy: Optional[torch.Tensor] = None, alpha0=None) -> torch.Tensor:
    return ResidualFn.apply(grid, q, xy, alpha0)


def forces(grid, q, xy: Optional[torch.Tensor] = None, alpha0=None) -> torch.Tensor:
    return ForceFn.apply(grid, q, xy, alpha0)


def steady_state(grid, q0, xy: Optional[torch.Tensor] = None, alpha0=None, n_iter: int = 1000,
                 n_adj_iter: Optional[int] = None) -> torch.Tensor:
    return SteadyStateFn.apply(grid, q0, xy, alpha0, int(n_iter),
                               int(n_iter if n_adj_iter is None else n_adj_iter))
