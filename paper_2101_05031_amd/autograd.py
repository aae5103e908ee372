"""torch.autograd.Function over the native field and its adjoint."""
from __future__ import annotations

import torch

from . import api


class SliceField(torch.autograd.Function):
    """field[nk, H, W] of planes [k0, k0+nk) as a differentiable function of
    the node positions [N,3] and strut weights [E].  The forward pass bins the
    lattice (nodes may have moved since the last call) and evaluates the
    field; the backward pass runs the native adjoint on the same bins.  When
    the weights are differentiated, struts of weight 0 are binned too, so
    their gradient is the true one rather than 0.
    support: optional per-strut supports [E] (held fixed)."""

    @staticmethod
    def forward(ctx, nodes, weight, edges, R, C, grid, k0, nk, tile=0, slab=0, support=None):
        # a weight of 0 still has a gradient (Eq. 6 is linear in the weight),
        # so when the weights are differentiated those struts stay binned
        bins = api.lattice_bin(nodes.detach().contiguous(), edges.contiguous(),
                               weight.detach().contiguous(), R, C, grid, tile=tile, slab=slab,
                               support=None if support is None else support.detach().contiguous(),
                               keep_zero_weight=bool(ctx.needs_input_grad[1]))
        field = api.slice_field(bins, k0, nk)
        ctx.bins = bins
        ctx.k0, ctx.nk = k0, nk
        return field

    @staticmethod
    def backward(ctx, grad):
        need_n, need_w = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_n or need_w):
            return (None,) * 11
        gw, gn = api.slice_field_backward(ctx.bins, ctx.k0, ctx.nk,
                                          grad.contiguous().to(ctx.bins.dtype),
                                          want_nodes=need_n)
        return (gn if need_n else None, gw if need_w else None,
                None, None, None, None, None, None, None, None, None)


def slice_field(nodes, weight, edges, R, C, grid, k0, nk, tile=0, slab=0, support=None):
    return SliceField.apply(nodes, weight, edges, R, C, grid, k0, nk, tile, slab, support)


def soft_occupancy_loss(field, target, C: float, tau: float):
    """sum over pixels of (sigmoid((g - C)/tau) - target)^2."""
    occ = torch.sigmoid((field - C) / tau)
    return ((occ - target) ** 2).sum()
