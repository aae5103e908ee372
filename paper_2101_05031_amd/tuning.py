"""Density matching by gradient descent on the strut weights (Sec. 5.3).

The paper matches per-voxel target densities by scaling the radii of a
tetrahedron's edges with a binary search, then refining with one common ratio
per voxel; the radii never drop below the smallest printable size.  Here every
strut weight is a free variable instead, moved by Adam along the gradient of a
smooth voxel-density loss:

    L(w) = sum_v (soft_density_v(w) - target_v)^2

with soft_density_v the per-voxel mean of sigmoid((g - C) / tau) over the
pixel-centre samples (slice_density_loss), and dL/dw from the field adjoint
(slice_field_backward).  Weights are clamped from below by w_min (the weight
of the thinnest printable strut).  Each iteration re-bins the lattice (the
strut boxes grow and shrink with the weights), evaluates the field of the
voxelised planes, the loss and its gradient, all in the native library; the
optimiser update is a handful of elementwise tensor operations.
"""
from __future__ import annotations

import math

import torch

from . import api


def match_density(nodes, edges, weight, R: float, C: float, grid, target, vx: int, vy: int,
                  vz: int, *, k0: int = 0, nk: int | None = None, tau: float = 0.05,
                  iters: int = 20, lr: float | None = None, w_min: float = 0.0,
                  betas=(0.9, 0.999), eps: float = 1e-12, tile: int = 0, slab: int = 0,
                  support=None, stream=None):
    """Adjust `weight` so the per-voxel densities of planes k0 .. k0+nk-1 move
    toward `target` (float32 [nz, ny, nx] on the device).

    support: optional per-strut supports [E], held fixed (the adjoint covers
    the quartic kernel only).

    lr defaults to 2% of the mean starting weight per step; it decays along a
    half cosine to a tenth of that over the iterations.  Returns (weight,
    history): the iterate with the lowest soft loss, and a list of dicts
    {loss, density_error} (the soft loss and the mean absolute error of the
    hard density, Eq. 9) for each iterate, the starting weights first and the
    last update's result last.
    """
    nk = grid.n_slices - k0 if nk is None else nk
    w = weight.detach().clone().contiguous()
    if lr is None:
        lr = 0.02 * float(w.mean())
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    b1, b2 = betas
    history = []

    def evaluate(w, want_grad):
        # struts at weight 0 stay binned: their gradient can move them back up
        bins = api.lattice_bin(nodes, edges, w, R, C, grid, tile=tile, slab=slab,
                               support=support, keep_zero_weight=True, stream=stream)
        field = api.slice_field(bins, k0, nk, stream=stream)
        loss, _, gfield = api.slice_density_loss(bins, field, target, tau, vx, vy, vz,
                                                 want_grad=want_grad, stream=stream)
        hard = api.slice_density(bins, field, vx, vy, vz, stream=stream)
        rec = {"loss": float(loss.item()),
               "density_error": float((hard - target).abs().mean().item())}
        gw = None
        if want_grad:
            gw, _ = api.slice_field_backward(bins, k0, nk, gfield, want_nodes=False,
                                             stream=stream)
        return rec, gw

    best_loss, best_w = math.inf, None
    for t in range(1, iters + 1):
        rec, g = evaluate(w, True)
        history.append(rec)
        if rec["loss"] < best_loss:
            best_loss, best_w = rec["loss"], w.clone()
        m.mul_(b1).add_(g, alpha=1.0 - b1)
        v.mul_(b2).addcmul_(g, g, value=1.0 - b2)
        lr_t = lr * (0.1 + 0.45 * (1.0 + math.cos(math.pi * (t - 1) / iters)))
        step = lr_t / (1.0 - b1 ** t)
        denom = (v / (1.0 - b2 ** t)).sqrt_().add_(eps)
        w.addcdiv_(m, denom, value=-step).clamp_(min=w_min)
    rec, _ = evaluate(w, False)
    history.append(rec)
    if rec["loss"] < best_loss:
        best_w = w
    return best_w, history
